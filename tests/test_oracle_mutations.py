"""The coupling pins catch plausible mistakes: each case plants one mistake in a copy of
the oracle's C source (a dropped term, a wrong sign, a wrong factor or distance),
compiles it on the CPU, and checks that the pin written for that part fails on it while
the unmodified oracle passes (test_oracle_coupling.py)."""
import os
import subprocess

import pytest

import coupling_pins as pins
import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "iblbm_ref.c")

# (name, text in the oracle, planted replacement, pin that must fail)
MUTATIONS = [
    ("load average dropped", "double Havg = 0.5 * (H + Hprev[a]);", "double Havg = H;",
     pins.pin_newton_euler_constant_loads),
    ("interior momentum change with the wrong sign", "double H = Fh[a] + (P[a] - Pprev[a]);",
     "double H = Fh[a] + (Pprev[a] - P[a]);", pins.pin_newton_euler_constant_loads),
    ("buoyant weight without the displaced fluid", "double meff = M - rho0 * V;",
     "double meff = M;", pins.pin_newton_euler_rigid_interior),
    ("angular velocity divided by the mass", "Om[a] = Om[a] + Gavg / I;",
     "Om[a] = Om[a] + Gavg / M;", pins.pin_newton_euler_constant_loads),
    ("position by explicit Euler", "X[a] = X[a] + 0.5 * (U0 + U1);", "X[a] = X[a] + U1;",
     pins.pin_newton_euler_constant_loads),
    ("indicator ramp shifted inward", "double chi = R + 0.5 - sqrt(d2);",
     "double chi = R - sqrt(d2);", pins.pin_interior_volume_and_moment),
    ("angular momentum cross product reversed",
     "double t[3] = {r[1] * m[2] - r[2] * m[1], r[2] * m[0] - r[0] * m[2], r[0] * m[1] - r[1] * m[0]};",
     "double t[3] = {r[2] * m[1] - r[1] * m[2], r[0] * m[2] - r[2] * m[0], r[1] * m[0] - r[0] * m[1]};",
     pins.pin_interior_volume_and_moment),
    ("torque added instead of subtracted", "T[a] = T[a] - t[a];", "T[a] = T[a] + t[a];",
     pins.pin_loads_closed_forms),
    ("point force not weighted by its shell volume",
     "double Fd[3] = {f[0] * dV[m], f[1] * dV[m], f[2] * dV[m]};",
     "double Fd[3] = {f[0], f[1], f[2]};", pins.pin_loads_closed_forms),
    ("wall image at distance h", "double d = 2.0 * h;", "double d = h;",
     pins.pin_wall_force_is_mirror_pair),
    ("wall force towards the wall", "Fc[3 * p + a] = Fc[3 * p + a] + (side == 0 ? mag : -mag);",
     "Fc[3 * p + a] = Fc[3 * p + a] + (side == 0 ? -mag : mag);", pins.pin_wall_force_is_mirror_pair),
    ("gap to the partner's centre minus its diameter", "double gg = sqrt(d2) - 0.5 * D[o];",
     "double gg = sqrt(d2) - D[o];", pins.pin_gap_feature_geometry),
    ("gap not clamped at zero", "return gap < 0.0 ? 0.0 : gap;", "return gap;",
     pins.pin_gap_feature_geometry),
    ("learned force without the previous step's",
     "F[3 * m + o] = o < dim ? Fprev[3 * m + o] + (tmean[o] + tsd[o] * y[NO * m + o]) : 0.0;",
     "F[3 * m + o] = o < dim ? (tmean[o] + tsd[o] * y[NO * m + o]) : 0.0;",
     pins.pin_learned_force_prediction),
    ("target mean and std swapped",
     "F[3 * m + o] = o < dim ? Fprev[3 * m + o] + (tmean[o] + tsd[o] * y[NO * m + o]) : 0.0;",
     "F[3 * m + o] = o < dim ? Fprev[3 * m + o] + (tsd[o] + tmean[o] * y[NO * m + o]) : 0.0;",
     pins.pin_learned_force_prediction),
    ("features not divided by their std",
     "xn[NI * m + i] = (feat[NI * m + i] - mean[i]) / sd[i];",
     "xn[NI * m + i] = feat[NI * m + i] - mean[i];", pins.pin_learned_force_prediction),
]


def _build_variant(tmp_path, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"the oracle no longer holds: {old}"
    path = tmp_path / "ref_variant.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / "libref_variant.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
                    "-Wno-unknown-pragmas", "-I", os.path.dirname(SRC), str(path), "-o", str(lib), "-lm"],
                   check=True)
    return oracle.load(str(lib))


@pytest.mark.parametrize("name,old,new,pin", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pin_catches_planted_mistake(tmp_path, name, old, new, pin):
    L = _build_variant(tmp_path, old, new)
    with pytest.raises(AssertionError):
        pin(L=L)
