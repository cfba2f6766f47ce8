"""Benchmark of the MI355X IB-LBM step: MLUPS on one GPU, the roofline fraction of the
dominant kernel, and the CPU oracle timed on the host beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A step is one pass of the whole hot path (band marking, cell list and pair forces, band
u*, the multi-direct-forcing passes, collide-stream, interior momentum, loads and
Newton-Euler) over the synthetic workload; inputs are resident in HBM before timing.
Prints one JSON line.  MLUPS = N_grid * steps / (1e6 * seconds) (the paper's Eq. 52).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix cores, published
# timed region: events on the dominant group's launches of every 5th step; the stride is
# odd, so the timed launches fall on both parities of the A-A streaming
TIMING_EVERY = 5
GROUPS = ["collide", "band", "interp", "spread", "interior", "particle", "mlp", "other"]
KERNEL_NAME = {"collide": "k_collide_stream", "band": "k_ustar_all",
               "interp": "k_interp_lds", "spread": "k_spread_lds",
               "interior": "k_interior", "particle": "k_cells + k_pairs + k_loads_newton",
               "mlp": "k_features + k_mlp_infer"}
# the kernel of a group whose counter traffic is recorded under profiles/
PMC_KERNEL = {"collide": "k_collide_stream", "band": "k_ustar_all", "interp": "k_interp_lds",
              "spread": "k_spread_lds", "interior": "k_interior", "particle": "k_pairs"}
# MLP 10-64-64-3: 2 (10*64 + 64*64 + 64*3) multiply-adds per point
MLP_FLOP_PER_POINT = 2 * (10 * 64 + 64 * 64 + 64 * 3)


def progress(msg):
    """a progress line on stderr (the JSON result stays alone on stdout)"""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(group, p, nmk, band_nodes, band_lattice=True):
    """Bytes one launch of a kernel group must move (f_0, padding and the method's own
    bookkeeping not credited):
      collide-stream   2 (q-1) s per node + d cs per band node (the force read)
      band u*          ((q-1) s + d cs) per band node
      interp + spread  per forcing pass 2 d cs per band node + 16 d per point (offsets in
                       FP64, U_b and dF); split as interpolation d cs per band node +
                       12 d per point (u read; offsets, U_b) and spreading d cs per band
                       node + 4 d per point (f update; dF)
    with s the stored PDF size and cs the compute size (4, and 8 in FP64).  Where the band
    u* is made inside the first of the mdf_iters interpolation launches (band_lattice
    false, a 2-D mode), each interpolation launch carries 1/mdf_iters of it."""
    dim = p["dim"]
    q = 9 if dim == 2 else 19
    s = {"f64": 8, "f32": 4, "bf16": 2, "f16": 2}[p["storage"]]
    cs = 8 if p["storage"] == "f64" else 4
    N = p["n"][0] * p["n"][1] * p["n"][2]
    band = ((q - 1) * s + dim * cs) * band_nodes
    if group == "collide":
        return 2 * (q - 1) * s * N + dim * cs * band_nodes
    if group == "band":
        return band
    if group == "interp":
        b = dim * cs * band_nodes + nmk * 12 * dim
        if not band_lattice:
            b += band / max(1, p["mdf_iters"])
        return b
    if group == "spread":
        return dim * cs * band_nodes + nmk * 4 * dim
    return None


def run(args):
    import numpy as np
    import torch

    from paper_2002_08855_amd import binding, inputs, traffic

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs an MI355X GPU")
    torch.cuda.set_device(0)
    w = inputs.workload(args.workload)
    p = dict(w["params"])
    p["stats_every"] = 0  # no slip statistic inside the timed region
    parts = w["particles"]
    sim = binding.Sim(p)
    if parts is not None:
        sim.add_particles(parts["center"], parts["diameter"], parts["density"],
                          n_markers=parts["n_markers"])
    np_, nmk = sim.counts()
    N = int(np.prod(p["n"]))
    sim.step(args.warmup)
    torch.cuda.synchronize()

    # per-group kernel-time breakdown (every group bracketed by HIP events)
    sim.set_timing(-1)
    sim.reset_stats()
    nb = max(5, min(args.steps, 50))
    sim.step(nb)
    st = sim.stats()
    per_group = {g: (st["time_ms"][g] / nb) for g in GROUPS if st["launches"][g]}
    dominant = max(per_group, key=per_group.get)
    band_nodes = st["band_nodes"]
    band_lattice = bool(st["band_lattice"])
    # the collide-stream kernel by itself (events with its launch), over the same steps
    sim.set_timing(1 << GROUPS.index("collide"))
    sim.set_timing_kernel(True)
    sim.reset_stats()
    sim.step(nb)
    st_c = sim.stats()
    sim.set_timing_kernel(False)

    # timed region: only the dominant group carries events (2 per launch), and only in
    # every TIMING_EVERY-th step, so that the events' own cost (an extra queue packet
    # each) stays out of the throughput
    sim.set_timing(1 << GROUPS.index(dominant))
    sim.set_timing_every(TIMING_EVERY)
    # the collide, interpolation and spreading kernels are timed on their own, with events
    # recorded as part of their launch (as the profiler times them)
    kernel_only = dominant in ("collide", "interp", "spread")
    sim.set_timing_kernel(kernel_only)
    sim.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st2 = sim.stats()
    sim.set_timing(0)
    sim.set_timing_every(1)
    sim.set_timing_kernel(False)
    secs = t1 - t0
    mlups = N * args.steps / (1e6 * secs)
    launches = st2["launches"][dominant]
    avg_ms = st2["time_ms"][dominant] / max(1, launches)
    nbytes = algorithmic_bytes(dominant, p, nmk, band_nodes, band_lattice)
    roof = None
    if nbytes is not None:
        ach = nbytes / (avg_ms * 1e-3) / 1e9
        roof = {"kernel": KERNEL_NAME.get(dominant, dominant), "bound": "hbm",
                "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                "avg_launch_ms": round(avg_ms, 5), "launches": launches,
                "timed_every_nth_step": TIMING_EVERY,
                "timing": "kernel execution (events with the launch)" if kernel_only
                          else "the group's launches between events",
                "algorithmic_bytes_per_launch": int(nbytes)}
        kname = PMC_KERNEL.get(dominant, dominant)
        prof = os.path.join(ROOT, "profiles", f"{kname}_{args.workload}_pmc.json")
        if os.path.exists(prof):
            d = json.load(open(prof))
            if d.get("source_sha") == traffic.source_sha(kname):
                roof["traffic"] = d.get("traffic_bytes_per_launch")
    # the collide-stream kernel against the HBM roofline
    roof_collide = None
    if st_c["launches"]["collide"]:
        nb_c = algorithmic_bytes("collide", p, nmk, band_nodes, band_lattice)
        ms_c = st_c["time_ms"]["collide"] / st_c["launches"]["collide"]
        ach_c = nb_c / (ms_c * 1e-3) / 1e9
        roof_collide = {"kernel": "k_collide_stream", "bound": "hbm", "achieved": round(ach_c, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(ach_c / HBM_PEAK_GBS, 4),
                        "avg_launch_ms": round(ms_c, 5), "algorithmic_bytes_per_launch": int(nb_c)}
    del sim
    torch.cuda.empty_cache()
    progress(f"{args.workload}: {mlups:.1f} MLUPS over {args.steps} steps")
    # the slip statistic needs particles; particle-free workloads report none
    slip_steps = int(w.get("steps", 500)) if args.slip_steps is None else args.slip_steps
    slip = slip_run(binding, w, slip_steps) if parts is not None and slip_steps > 0 else None
    out = {
        "metric": "MLUPS at phi=0.40 (plain FP32 vs BF16-PDF / learned forcing) at stated slip error",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * secs / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"f64": "f64", "f32": "f32", "bf16": "bf16-storage/f32", "f16": "f16-storage/f32"}[
            p["storage"]],
        "data": "synthetic",
        "config": {"workload": args.workload, "n": list(p["n"][:p["dim"]]), "particles": np_,
                   "points_per_particle": (parts or {}).get("n_markers", 0),
                   "mdf_iters": p["mdf_iters"], "storage": p["storage"], "tau": p["tau"],
                   "parallelism": "1 GPU"},
        "slip_rms": slip["slip_rms"] if slip else None,
        "slip": slip,
        "roofline": roof,
        "roofline_collide_stream": roof_collide,
        "kernel_ms_per_step": {g: round(v, 5) for g, v in per_group.items()},
    }
    if not args.no_forms:
        out["forms"] = run_forms(args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, args)
    return out


def slip_run(binding, w, steps, params=None, mlp=None):
    """The slip error: the rms of |U_b - D_I u| over the points after the step's final
    forcing pass, averaged over the last half of a run of `steps` steps from the
    workload's initial state."""
    import numpy as np

    p = dict(params if params is not None else w["params"])
    p["stats_every"] = 0
    parts = w["particles"]
    sim = _sim(binding, p, parts)
    if mlp is not None:
        sim.set_mlp(*mlp)
    first = steps // 2
    sim.step(first)
    sim.set_stats_every(1)
    vals = []
    for _ in range(steps - first):
        sim.step(1)
        vals.append(sim.stats()["slip_rms"])
    fb = sim.stats()["fallbacks"]
    umax = float(np.abs(sim.particles()["U"]).max())
    del sim
    vals = np.array(vals)
    return {"slip_rms": float(vals.mean()), "slip_rms_last": float(vals[-1]),
            "steps": steps, "averaged_steps": int(len(vals)), "fallbacks": int(fb),
            "max_abs_U_end": umax}


def _timed(sim, N, steps, warmup):
    """MLUPS over `steps` after `warmup` (no slip statistic inside the timed steps)"""
    import torch

    sim.set_stats_every(0)
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    return {"value": round(N * steps / (1e6 * secs), 1), "ms_per_step": round(1e3 * secs / steps, 4),
            "steps": steps, "warmup": warmup}


def _sim(binding, p, parts):
    sim = binding.Sim(p)
    sim.add_particles(parts["center"], parts["diameter"], parts["density"],
                      n_markers=parts["n_markers"])
    return sim


def _breakdown(sim, steps=10):
    """kernel-group times per step (every group bracketed by HIP events)"""
    sim.set_stats_every(0)
    sim.set_timing(-1)
    sim.reset_stats()
    sim.step(steps)
    st = sim.stats()
    sim.set_timing(0)
    return {g: round(st["time_ms"][g] / steps, 5) for g in GROUPS if st["launches"][g]}


def run_forms(args, only=None):
    """The other forms of the step on their workloads:
    - PDFs stored as BF16 (384^3, 25033 spheres, volume fraction 0.40);
    - the paper's single-pass thickened-shell forcing against plain MDF-3 (2048^2, 4096
      disks);
    - learned forcing (256^3, 2347 spheres, 0.30) against plain MDF-5 and against MDF-2,
      the plain method with the same number of spreading passes.  The network is trained
      here, on the GPU, on (features, converged MDF-5 force) pairs captured from plain runs
      of two other packings (cavity256_train: 1565 spheres, 0.20, random addition;
      cavity256_train30: 2347 spheres, 0.30, a finer FCC lattice; each with its own seed),
      so the evaluation set is held out.
    Each form reports MLUPS over timed steps and the slip averaged over the last half of
    a run of the workload's length.  `only` names one form to run by itself (for a
    profiler run)."""
    import numpy as np
    import torch

    from paper_2002_08855_amd import binding, inputs

    forms = {}
    steps, warmup = args.form_steps, 3

    def measure(w, name, params=None, mlp=None):
        p = dict(params if params is not None else w["params"])
        sim = _sim(binding, p, w["particles"])
        if mlp is not None:
            sim.set_mlp(*mlp)
        r = _timed(sim, int(np.prod(p["n"])), steps, warmup)
        r["kernel_ms_per_step"] = _breakdown(sim)
        np_, nmk = sim.counts()
        del sim
        torch.cuda.empty_cache()
        n_slip = int(w.get("steps", 200)) if args.slip_steps is None else args.slip_steps
        r["slip"] = slip_run(binding, w, n_slip, params=p, mlp=mlp) if n_slip > 0 else None
        r["slip_rms"] = r["slip"]["slip_rms"] if r["slip"] else None
        r.update({"workload": name, "particles": np_, "points": nmk})
        return r

    def bf16_storage():
        r = measure(inputs.workload("cavity384_bf16"), "cavity384_bf16")
        r["dtype"] = "bf16-storage/f32"
        return r

    def btdf_single_pass():
        # the paper's own coupling for its particle-laden runs: one forcing pass with the
        # shell thickened to drs = 1.9 (3-point kernel), against plain MDF-3 with the
        # 4-point kernel, on the same lattice and particles (the sparse 2-D layout: at the
        # dense workloads' near contacts the single thickened pass does not settle stably)
        res = {}
        for name in ("cavity2048_sparse", "cavity2048_sparse_btdf"):
            w = inputs.workload(name)
            p = w["params"]
            res[name] = measure(w, name)
            res[name].update({"delta": ["peskin4", "roma3"][p["delta"]], "drs": p["drs"],
                              "mdf_iters": p["mdf_iters"], "dtype": "f32"})
        r = dict(res["cavity2048_sparse_btdf"])
        r["plain_mdf3"] = res["cavity2048_sparse"]
        return r

    def learned_forcing():
        return learned_form(binding, inputs, measure, warmup)

    for name, fn in (("bf16_storage", bf16_storage), ("btdf_single_pass", btdf_single_pass),
                     ("learned_forcing", learned_forcing)):
        if only not in (None, name):
            continue
        try:
            forms[name] = fn()
        except Exception as e:  # reported, not fatal for the headline line
            forms[name] = {"error": repr(e)}
        progress(f"form {name} done")
    return forms


def learned_form(binding, inputs, measure, warmup):
    """Train on captures of plain MDF-5 runs of two other packings (cavity256_train and
    cavity256_train30), evaluate on cavity256_learned, held out: learned + 1 correction
    pass, plain MDF-5 and plain MDF-2."""
    import numpy as np

    # captures spread over the same 200 steps from rest that the evaluation run covers,
    # from two training packings (0.20 by random addition, 0.30 on a finer FCC lattice)
    feats, tgts = [], []
    train_sets = ("cavity256_train", "cavity256_train30")
    for name in train_sets:
        wt = inputs.workload(name)
        sim = _sim(binding, wt["params"], wt["particles"])
        for _ in range(10):
            sim.step(20)
            f, t = sim.capture_samples()
            feats.append(f)
            tgts.append(t)
        del sim
    f = np.concatenate(feats)
    t = np.concatenate(tgts)
    # the network's target: the change of the converged force over the previous step's
    r = t - f[:, 3:6]
    norm = np.concatenate([f.mean(0), f.std(0) + 1e-12, r.mean(0), r.std(0) + 1e-12])
    xn = (f - norm[:10]) / norm[10:20]
    tn = (r - norm[20:23]) / norm[23:26]
    P0 = np.random.default_rng(1).normal(0, 0.1, binding.NPARAM)
    epochs = 8
    progress(f"learned form: {len(f)} training samples captured")
    t0 = time.perf_counter()
    P, curve = binding.nn_train(xn, tn, P0, epochs=epochs, batch=8192, lr=2e-3, seed=1)
    progress(f"learned form: trained in {time.perf_counter() - t0:.1f} s")
    train_s = time.perf_counter() - t0
    w = inputs.workload("cavity256_learned")
    base = dict(w["params"])
    rl = measure(w, "cavity256_learned", params=base, mlp=(P, norm))
    rp5 = measure(w, "cavity256_learned", params=dict(base, forcing=0, mdf_iters=5))
    rp2 = measure(w, "cavity256_learned", params=dict(base, forcing=0, mdf_iters=2))
    # the MLP kernels (features + BF16 MFMA inference) against the dense BF16 peak
    t_mlp = rl["kernel_ms_per_step"].get("mlp")
    if t_mlp:
        flops = rl["points"] * MLP_FLOP_PER_POINT
        rl["mlp_mfma"] = {"kernels": "k_features + k_mlp_infer", "ms_per_step": t_mlp,
                          "flop_per_step": flops,
                          "achieved_tflops": round(flops / (t_mlp * 1e-3) / 1e12, 3),
                          "peak_tflops": BF16_MFMA_PEAK_TFLOPS,
                          "frac": round(flops / (t_mlp * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFLOPS, 6)}
    rl.update({"dtype": "f32, MLP in bf16 on MFMA", "correction_passes": 1,
               "train": {"workloads": list(train_sets), "samples": int(len(f)),
                         "captures": len(feats), "epochs": epochs,
                         "seconds": round(train_s, 2), "loss_first": float(curve[0]),
                         "loss_last": float(curve[-1])},
               "plain_mdf5": rp5, "plain_mdf2": rp2})
    return rl


SWEEP = {2: [40, 100, 200, 400, 1000, 2000, 4000, 8192], 3: [40, 80, 128, 160, 210, 256, 384, 480]}


def run_sweep(args):
    """The particle-free channel of Sec. 6.1 (inflow and outflow faces by non-equilibrium
    extrapolation) at the paper's domain sizes and beyond, FP32: MLUPS against the number
    of nodes, and the collide-stream rate against the HBM peak."""
    import numpy as np
    import torch

    from paper_2002_08855_amd import binding, inputs

    rows = []
    for dim in (2, 3):
        q = 9 if dim == 2 else 19
        for n in SWEEP[dim]:
            w = inputs.workload(f"channel{dim}d_{n}")
            p = w["params"]
            N = int(np.prod(p["n"]))
            sim = binding.Sim(p)
            steps = int(max(20, min(2000, 4e9 / N)))
            r = _timed(sim, N, steps, 10)
            bytes_per_node = 2 * (q - 1) * 4
            gbs = r["value"] * 1e6 * bytes_per_node / 1e9
            rows.append({"dim": dim, "n": n, "nodes": N, "mlups": r["value"], "ms_per_step": r["ms_per_step"],
                         "steps": steps, "step_gbs": round(gbs, 1), "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
            del sim
            torch.cuda.empty_cache()
    return {"sweep": "channel (Sec. 6.1), FP32, whole step", "unit": "MLUPS", "rows": rows}


NP_SWEEP = {2: [1, 10, 100, 1000, 5000, 10000], 3: [1, 10, 100, 300, 600]}
RES_SWEEP = {2: [12, 16, 24, 32, 40, 48], 3: [12, 16, 20, 24, 30]}


def run_np_sweep(args, kind="np", suffix=""):
    """The particle-count series of Table 7 (Sec. 6.2.1; kind "np": 2048^2 with D = 16,
    150^3 with D = 12) or the resolution series of Sec. 6.2.2 (kind "res": a 40 D square
    with 400 disks, a 5 D cube with 27 spheres): whole-step MLUPS and the time of each
    kernel group per step (FP32, MDF-3)."""
    import numpy as np
    import torch

    from paper_2002_08855_amd import binding, inputs

    rows = []
    series = NP_SWEEP if kind == "np" else RES_SWEEP
    for dim in (2, 3):
        for v in series[dim]:
            w = inputs.workload(f"{kind}{dim}d_{v}{suffix}")
            p, parts = w["params"], w["particles"]
            N = int(np.prod(p["n"]))
            sim = _sim(binding, p, parts)
            steps = 100 if dim == 2 else 50
            r = _timed(sim, N, steps, 5)
            sim.set_stats_every(0)
            sim.set_timing(-1)
            sim.reset_stats()
            sim.step(20)
            st = sim.stats()
            sim.set_timing(0)
            groups = {g: round(st["time_ms"][g] / 20, 5) for g in GROUPS if st["launches"][g]}
            np_, nmk = sim.counts()
            del sim
            torch.cuda.empty_cache()
            # the paper's run length (1000 steps in 2-D, 200 in 3-D), from rest: slip over
            # its last half, and the largest particle speed at its end
            slip = slip_run(binding, w, int(w.get("steps", 200)))
            rows.append({"dim": dim, "n": list(p["n"][:dim]), "diameter": float(parts["diameter"][0]),
                         "particles": np_, "points": nmk, "density_ratio": float(parts["density"][0]),
                         "mesh_ratio": round(nmk / N, 6), "mlups": r["value"],
                         "ms_per_step": r["ms_per_step"], "slip_rms": slip["slip_rms"],
                         "run_steps": slip["steps"], "max_abs_U_end": slip["max_abs_U_end"],
                         "kernel_ms_per_step": groups})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    what = "particle count (Table 7)" if kind == "np" else "particle resolution (Sec. 6.2.2)"
    how = ("3-point kernel, drs 1.9, one forcing pass, density ratio 1.01 (Sec. 6.2)"
           if suffix else "MDF-3, 4-point kernel, density ratio 1.5")
    return {"sweep": f"{what}, FP32, {how}", "unit": "MLUPS", "rows": rows}


CPU_CHILD = r"""
import json, os, sys, time
sys.path.insert(0, ROOT)
if PIN is not None:
    os.sched_setaffinity(0, {PIN})
import numpy as np
import oracle
from paper_2002_08855_amd import inputs
w = inputs.workload(WORKLOAD)
p, parts = w["params"], w["particles"]
s = oracle.Sim(p)
if parts is not None:
    s.add_particles(parts["center"], parts["diameter"], parts["density"], n_markers=parts["n_markers"])
s.step(1)  # warm
steps, t = 0, 0.0
while t < BUDGET and steps < 1000:
    t0 = time.perf_counter()
    s.step(1)
    t += time.perf_counter() - t0
    steps += 1
print(json.dumps({"steps": steps, "seconds": t, "N": int(np.prod(p["n"]))}))
"""


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_leg(workload, threads, pin, budget):
    import subprocess

    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    code = (f"ROOT = {ROOT!r}\nWORKLOAD = {workload!r}\nBUDGET = {budget!r}\nPIN = {pin!r}\n"
            + CPU_CHILD)
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       timeout=600)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-2000:])
    d = json.loads(r.stdout.strip().splitlines()[-1])
    return d


def cpu_baseline(w, args):
    """The CPU oracle (FP64, OpenMP over lattice loops) on a bounded sample of the same
    workload (the same lattice and particles, the steps that fit the time budget after one
    warm-up step), in two child processes: all the host cores this process may use (at
    most 16), and one thread pinned to one core (the paper's setting is one core)."""
    import oracle

    allowed = sorted(os.sched_getaffinity(0))
    threads = min(16, len(allowed))
    legs = {}
    for key, nthr, pin in (("all_cores", threads, None), ("single_core", 1, allowed[0])):
        d = _cpu_leg(args.workload, nthr, pin, args.cpu_seconds)
        legs[key] = {"value": round(d["N"] * d["steps"] / (1e6 * d["seconds"]), 3),
                     "unit": "MLUPS", "cores": nthr,
                     "sample": f"{d['steps']} steps of {args.workload} after 1 warm-up step "
                               f"({d['seconds']:.1f} s), FP64 oracle, OMP_NUM_THREADS={nthr}"
                               + (f", pinned to CPU {pin}" if pin is not None else "")}
    out = dict(legs["all_cores"])
    out.update({"kind": "oracle", "single_core": legs["single_core"], "cpu_model": _cpu_model(),
                "host_cpus_allowed": len(allowed),
                "compiler": f"{oracle.compiler_version()} {' '.join(oracle.CFLAGS)}"})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cavity2048_f32")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the BF16-storage and learned-forcing forms")
    ap.add_argument("--form-steps", type=int, default=20)
    ap.add_argument("--slip-steps", type=int, default=None,
                    help="length of the run the slip is averaged over (default: the "
                         "workload's run length; 0 skips it, e.g. under a profiler)")
    ap.add_argument("--form", choices=["bf16_storage", "btdf_single_pass", "learned_forcing"],
                    help="instead of the headline line: run one form by itself")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the headline line: MLUPS of the particle-free channel "
                         "(inflow/outflow faces) against the domain size")
    ap.add_argument("--np-sweep", action="store_true",
                    help="instead of the headline line: MLUPS and kernel-group times against "
                         "the number of particles (Table 7)")
    ap.add_argument("--np-sweep-paper", action="store_true",
                    help="the particle-count series in the paper's setting (3-point kernel, "
                         "drs 1.9, one forcing pass, density ratio 1.01)")
    ap.add_argument("--res-sweep", action="store_true",
                    help="instead of the headline line: the same against the particle "
                         "resolution (Sec. 6.2.2)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the IB-LBM step runs on one GPU; --gpus above 1 is not "
                                   "supported (the multi-GPU slab decomposition is not built)"}))
        sys.exit(2)
    if args.sweep:
        print(json.dumps(run_sweep(args)), flush=True)
        return
    if args.np_sweep:
        print(json.dumps(run_np_sweep(args)), flush=True)
        return
    if args.np_sweep_paper:
        print(json.dumps(run_np_sweep(args, suffix="_paper")), flush=True)
        return
    if args.res_sweep:
        print(json.dumps(run_np_sweep(args, "res")), flush=True)
        return
    if args.form:
        print(json.dumps(run_forms(args, only=args.form)), flush=True)
        return
    out = run(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
