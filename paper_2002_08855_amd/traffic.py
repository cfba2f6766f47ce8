"""HBM traffic of one kernel from rocprofv3 counters, scaled by a plain copy kernel.

Two steps, both run by hand:

1. Under ``rocprofv3 --pmc FETCH_SIZE`` (and once more under ``--pmc WRITE_SIZE``), run

       python -m paper_2002_08855_amd.traffic run --workload NAME --steps K

   It first launches a plain elementwise copy of a known size (COPY_BYTES read and
   COPY_BYTES written), then K steps of the workload.

2. Reduce the two counter CSVs to bytes per launch of one kernel:

       python -m paper_2002_08855_amd.traffic reduce --fetch DIR --write DIR \\
           --workload NAME --kernel k_spread_lds --out profiles/NAME.json

   FETCH_SIZE and WRITE_SIZE are reported in KiB per dispatch; each is scaled by the
   ratio of the copy's known bytes to what the same counter read for the copy.  The
   result records a hash of the kernel's source and of the host code that launches it,
   so that a reader can tell when it no longer describes the built kernel.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
COPY_BYTES = 1 << 30
SOURCE_OF = {"k_collide_stream": "lbm.hip", "k_interior": "lbm.hip", "k_interp_lds": "ibm.hip",
             "k_spread_lds": "ibm.hip", "k_band_prep": "ibm.hip", "k_ustar_all": "lbm.hip",
             "k_pairs": "particles.hip",
             "k_cells": "particles.hip", "k_loads_newton": "particles.hip",
             "k_features": "mlp.hip", "k_mlp_infer": "mlp.hip"}


def source_sha(kernel):
    """hash of the kernel's source file, the headers every kernel includes and the host
    code that sets the launch shapes and work units"""
    h = hashlib.sha256()
    for f in (SOURCE_OF[kernel], "common.h", "pdf_access.h", "index_math.h", "host.hip"):
        h.update(open(os.path.join(ROOT, "paper_2002_08855_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def run(args):
    import torch

    from paper_2002_08855_amd import binding, inputs

    a = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    w = inputs.workload(args.workload)
    p = dict(w["params"])
    parts = w["particles"]
    sim = binding.Sim(p)
    if parts is not None:
        sim.add_particles(parts["center"], parts["diameter"], parts["density"],
                          n_markers=parts["n_markers"])
    if p.get("forcing") == 1:
        # the learned form: the bytes the MLP kernels move do not depend on the weights
        import numpy as np

        P = np.random.default_rng(0).normal(0.0, 0.1, binding.NPARAM)
        norm = np.concatenate([np.zeros(10), np.ones(10), np.zeros(3), np.full(3, 1e-6)])
        sim.set_mlp(P, norm)
    sim.step(args.steps)
    torch.cuda.synchronize()
    print(json.dumps({"workload": args.workload, "steps": args.steps}), flush=True)


def _rows(d):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    out = []
    for f in files:
        with open(f) as fh:
            out.extend(csv.DictReader(fh))
    return out


def _per_dispatch(rows, counter):
    """{dispatch id: (kernel name, value)} summed over the counter's instances"""
    acc = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        k = r.get("Dispatch_Id") or r.get("Correlation_Id")
        name = r.get("Kernel_Name", "")
        v = float(r["Counter_Value"])
        if k in acc:
            acc[k] = (name, acc[k][1] + v)
        else:
            acc[k] = (name, v)
    return acc


def _mean_for(acc, pred):
    vals = [v for name, v in acc.values() if pred(name)]
    if not vals:
        return None, 0
    return sum(vals) / len(vals), len(vals)


def reduce_(args):
    fetch = _per_dispatch(_rows(args.fetch), "FETCH_SIZE")
    write = _per_dispatch(_rows(args.write), "WRITE_SIZE")
    is_copy = lambda n: "MulFunctor" in n  # the copy b = a * 1 of COPY_BYTES
    is_k = lambda n: args.kernel in n
    cf, ncf = _mean_for(fetch, is_copy)
    cw, ncw = _mean_for(write, is_copy)
    kf, nkf = _mean_for(fetch, is_k)
    kw, nkw = _mean_for(write, is_k)
    if None in (cf, cw, kf, kw):
        raise SystemExit("copy kernel or target kernel missing from the counter files")
    sf = COPY_BYTES / (cf * 1024.0)
    sw = COPY_BYTES / (cw * 1024.0)
    res = {
        "kernel": args.kernel, "workload": args.workload,
        "source_sha": source_sha(args.kernel),
        "fetch_kib_per_launch": kf, "write_kib_per_launch": kw, "launches": [nkf, nkw],
        "copy_bytes": COPY_BYTES, "copy_fetch_kib": cf, "copy_write_kib": cw,
        "scale_fetch": sf, "scale_write": sw,
        "traffic_bytes_per_launch": int(kf * 1024.0 * sf + kw * 1024.0 * sw),
        "commands": [
            f"rocprofv3 --pmc {c} -f csv -d <dir> -o run -- python -m paper_2002_08855_amd.traffic "
            f"run --workload {args.workload} --steps {args.steps}" for c in ("FETCH_SIZE", "WRITE_SIZE")
        ] + [f"python -m paper_2002_08855_amd.traffic reduce --fetch <dir> --write <dir> "
             f"--workload {args.workload} --kernel {args.kernel} --steps {args.steps} "
             f"--out profiles/{args.kernel}_{args.workload}_pmc.json"],
    }
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)
    print(json.dumps(res))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--workload", required=True)
    r.add_argument("--steps", type=int, default=3)
    d = sub.add_parser("reduce")
    d.add_argument("--fetch", required=True)
    d.add_argument("--write", required=True)
    d.add_argument("--workload", required=True)
    d.add_argument("--kernel", required=True)
    d.add_argument("--out", required=True)
    d.add_argument("--steps", type=int, default=3, help="steps of the counted run (recorded)")
    args = ap.parse_args(argv)
    if args.cmd == "run":
        run(args)
    else:
        reduce_(args)


if __name__ == "__main__":
    sys.exit(main())
