"""Benchmark of the nonconforming multiple-traces BEM hot path on one MI355X.

One step = one pass of the whole path on the FP64 workload "sphere-ico4/fib2002"
(unit sphere; exterior icosphere level 4, 5120 triangles / 2562 nodes;
interior independent Fibonacci grid 4000 triangles / 2002 nodes, rotated and
jittered 2 %; k_ext 5, k_int 8, rho_int/rho_ext 1.5; one plane wave; GMRES
tol 1e-6): mesh tables, dense V/K/T/D on both meshes (regular + singular
quadrature), mass and mortar matrices, dense inverse masses, load vector,
unrestarted GMRES on the mass-preconditioned system, traces back to the host
numbering.  value = dense entries assembled (4 N_e^2 + 4 N_i^2 per step) per
second of whole-step wall time (Gentries/s).
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP64_VEC_TFLOPS = 78.6       # MI355X FP64 vector


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU row sharding is a design note, not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2206_00708_amd as B
    import synth

    c = synth.make_config("C2")
    (xe, te), (xi, ti) = c["ext"], c["int"]
    ne, ni = len(xe), len(xi)
    entries = 4 * ne * ne + 4 * ni * ni
    torch.cuda.init()
    ctx = B.Context(0)
    stream = ctx.stream

    def step():
        me, mi = B.Mesh(ctx, xe, te), B.Mesh(ctx, xi, ti)
        p = B.Problem(ctx, me, mi, c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"])
        t0 = time.perf_counter()
        p.assemble_operators()
        torch.cuda.synchronize()
        t_asm = time.perf_counter() - t0
        p.assemble_projection()
        out, stats, code = p.solve(c["dirs"], tol=c["tol"], maxit=3000)
        x = out.cpu().numpy()
        return p, x, stats, code, t_asm

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lat, asm, iters = [], [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        t0 = time.perf_counter()
        p, x, stats, code, t_asm = step()
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
        asm.append(t_asm)
        iters.append(stats["iterations"])
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start

    value = entries * args.steps / total / 1e9
    line = {
        "metric": "dense BEM assembly Gentries/s; solves/s vs plain FP64 at 1e-5 err; p99 latency",
        "value": round(value, 4),
        "unit": "Gentries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "sphere-ico4/fib2002 MTF, FP64, 1 plane wave, GMRES tol 1e-6",
                   "n_ext": ne, "n_int": ni, "k_ext": c["k_ext"], "k_int": c["k_int"],
                   "rho_ratio": c["rho_int"] / c["rho_ext"], "parallelism": "single GPU"},
        "assembly_gentries_per_s": round(entries / statistics.median(asm) / 1e9, 3),
        "solves_per_s": round(args.steps / total, 3),
        "p50_ms": round(1e3 * statistics.median(lat), 3),
        "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 3),
        "gmres_iterations": int(statistics.median(iters)),
        "t_regular_ms": round(stats["t_regular_ms"], 3),
        "t_singular_ms": round(stats["t_singular_ms"], 3),
        "t_projection_ms": round(stats["t_projection_ms"], 3),
        "t_solve_ms": round(stats["t_solve_ms"], 3),
        "t_iter_ms": round(stats["t_iter_ms"], 4),
        "rel_residual": stats["rel_residual"],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
