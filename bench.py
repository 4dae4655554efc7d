"""Benchmark of the nonconforming multiple-traces BEM hot path on one MI355X.

One step = one pass of the whole path on the headline workload
"ellipsoid-ico5/fib8002" in FP64 (complex128, the precision of the paper's
dense operators): ellipsoid with semi-axes (1, 0.8, 0.6); exterior
icosphere level 5 (20,480 triangles, 10,242 nodes); interior independent
Fibonacci grid (16,000 triangles, 8,002 nodes), rotated and jittered 1 %;
k_ext 10, k_int 20, rho_int/rho_ext 2; one plane wave; GMRES to 1e-7 (the
tolerance at which the traces lie within 1e-5 of the exact discrete
solution).  The step covers mesh tables, dense V/K/T/D on both meshes
(regular + singular quadrature), mass and mortar matrices and the inverse
mass set-up, the load vector, unrestarted GMRES on the mass-preconditioned
system and the traces in the caller's numbering (left in device memory; the
mesh arrays are host inputs of about 1 MB).

value = dense entries assembled (4 N_e^2 + 4 N_i^2 per step) per second of
whole-step wall time, in Gentries/s.  The line also carries assembly-only
Gentries/s, solves/s, p50/p99 step latency, a per-phase breakdown, the trace
error against the oracle's exact discrete solution (tests/golden), the
roofline of the dominant kernel (timed with HIP events on the library's
stream during the timed steps), the FP64 CPU oracle timed on a bounded
sample of the same operators, and further objects: `c2` (the smaller FP64
sphere workload), `precision` (the mixed form on the headline workload),
`batching` (64 plane waves in one block solve vs one-at-a-time solves, with
the matrix-core roofline), `serving` (a seeded Poisson stream through the
request loop), and the exterior formulations, field, mortar and incident
variations.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
FP64_VEC_TFLOPS = 78.6       # MI355X FP64 vector, TFLOP/s

# Algorithmic FP64 work per quadrature point pair of the regular kernel,
# counting a fused multiply-add as two flops (as the vector peak does):
# difference and squared distance 8, 1/r and r 2, phase k r 1, reduction by
# pi/2 and the sin/cos polynomials 46, exp(ikr)/r 2, its radial derivative 7,
# the two normal projections 10 and their products 4, accumulation of the
# three 3-vectors of partial sums and of sum G 40, and the share of the
# per-row contraction 19.
FLOP_PER_POINT_PAIR = 139

# GMRES tolerance of each headline workload: at the workload's own 1e-6 the
# C3 traces can sit up to about 1.5e-5 from the exact discrete solution, at
# 1e-7 within 1e-6 (tests/golden; the bench reports the error it measures).
HEADLINE_TOL = {"C3": 1e-7, "C2": 1e-6}

# HBM traffic per launch of the dominant kernel from the FETCH_SIZE and
# WRITE_SIZE counters (rocprofv3 --pmc, one counter per run), each scaled by
# the counter's reading for a plain 1 GiB device copy (FETCH x 2.000, WRITE x
# 1.000), per workload, with the sha1 of the kernel's source text (the
# regions of solve.hip between the markers: its device helpers and the
# symmetric tile kernel) that the counters were taken on; the figure is
# reported only while that text is unchanged.
MTF_REGIONS = {"source": "paper_2206_00708_amd/csrc/solve.hip",
               "regions": [("namespace {", "}  // namespace"),
                           ("// ---- symmetric tile form", "// y rows = sum of the tile partials")]}
COUNTED_TRAFFIC = {
    ("mtf_dense", "C3"): {"bytes": 2.000 * 2669427.6 * 1024 + 1.000 * 47448.1 * 1024,
                          "sha1": "622b2e5ac6d2f07a3f71f5aa39f9288938c00ba8", **MTF_REGIONS},
}

# FP64 VALU counters of the regular-pair kernel per launch (rocprofv3 --pmc,
# kernels serialised by the counter collection), per workload, with the sha1
# of the regular-pair region of assemble.hip they were taken on (from the
# section's opening marker to the gather's): FP64 flops (SQ_INSTS_VALU_FLOPS_FP64 x
# 64 lanes), VALU instructions (SQ_INSTS_VALU), the VALU issue fraction
# (SQ_INSTS_VALU x 4 cycles over the SIMD cycles of the launch, from
# GRBM_GUI_ACTIVE per XCD x 1024 SIMDs) and the share of the FP64 flops in
# the software sin/cos (the small-angle polynomials and the rotation by the
# pair's base phase: 46 of the per-point-pair flops).
REG_REGIONS = {"source": "paper_2206_00708_amd/csrc/assemble.hip",
               "regions": [("// ------------------------------------------------------------ regular pairs",
                            "// The contributions to dense entry (i, j) of the tiles of one strip")]}
COUNTED_VALU = {
    ("regular_tiles", "C3"): {"flops_fp64": 1310718788.0 * 64, "valu_insts": 1067106586, "valu_busy": 0.701,
                              "sincos_flop_share": 0.32, "isolated_launch_us": 2715.7,
                              "sha1": "25fb264f3ef5797c79b384c65d0d644e4e7ed33b", **REG_REGIONS},
    ("regular_tiles", "C2"): {"flops_fp64": 864256332.0 * 64, "valu_insts": 702649931, "valu_busy": 0.704,
                              "sincos_flop_share": 0.32, "isolated_launch_us": 1912.8,
                              "sha1": "25fb264f3ef5797c79b384c65d0d644e4e7ed33b", **REG_REGIONS},
}


def kernel_source_sha1(t):
    import hashlib
    with open(os.path.join(ROOT, t["source"])) as f:
        text = f.read()
    h = hashlib.sha1()
    for a, b in t.get("regions", [(None, None)]):
        if a is None:
            h.update(text.encode())
            continue
        i = text.index(a)
        h.update(text[i:text.index(b, i)].encode())
    return h.hexdigest()


def counted_traffic(kernel, workload):
    t = COUNTED_TRAFFIC.get((kernel, workload))
    if not t or kernel_source_sha1(t) != t["sha1"]:
        return None
    return round(t["bytes"])


def counted_valu(kernel, workload, launch_ms):
    """FP64 rate of the kernel by its counted FLOPs per launch over the live
    average launch duration, with the counters' VALU busy fraction."""
    t = COUNTED_VALU.get((kernel, workload))
    if not t or kernel_source_sha1(t) != t["sha1"]:
        return None
    ach = t["flops_fp64"] / (launch_ms * 1e-3) / 1e12
    iso = t["flops_fp64"] / (t["isolated_launch_us"] * 1e-6) / 1e12
    return {"flops_fp64_per_launch": t["flops_fp64"], "achieved": round(ach, 2), "peak": FP64_VEC_TFLOPS,
            "frac": round(ach / FP64_VEC_TFLOPS, 4), "valu_busy": t["valu_busy"],
            "valu_insts_per_launch": t["valu_insts"], "sincos_flop_share": t.get("sincos_flop_share"),
            "isolated": {"launch_us": t["isolated_launch_us"], "achieved": round(iso, 2),
                         "frac": round(iso / FP64_VEC_TFLOPS, 4),
                         "note": "launch duration under the counter run, kernels serialised (no gather beside it)"}}


def golden(name):
    """The oracle's exact discrete solution of a workload (tests/golden, written
    by tests/golden/make_mtf_traces.py from the oracle alone), or None."""
    import numpy as np
    path = os.path.join(ROOT, "tests", "golden", f"mtf_{name}.npz")
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        return z["x"].astype(np.complex128)


def trace_error(x, ref, ne, ni):
    """Largest relative l2 error over the four trace blocks [v_e, w_e, v_i, w_i]."""
    import numpy as np
    cuts = [0, ne, 2 * ne, 2 * ne + ni, 2 * ne + 2 * ni]
    return max(float(np.linalg.norm(x[a:b] - ref[a:b]) / np.linalg.norm(ref[a:b])) for a, b in zip(cuts, cuts[1:]))


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_oracle_baseline(c, budget_s=15.0):
    """The FP64 oracle on the host cores, on bounded samples of the headline
    workload: assembly throughput (rows of V/K/T/D of both meshes) with all
    threads and with one, and the dense multiple-traces mat-vec (the oracle's
    matrix-vector product, numpy) on a block of rows of the printed system
    (the sampled interior rows: [-P_ie / 2, 0, -K_i, V_i] and
    [0, -c P_ie / 2, D_i, T_i], repeated to 1024 rows).  The oracle's full solve (assembly and
    dense LU) is quoted from the golden run's record, which states its host."""
    import json as _json
    import numpy as np
    from oracle import oracle as O
    O.lib()
    threads = O.max_threads()
    rng = np.random.default_rng(0)
    (xe, te), (xi, ti) = c["ext"], c["int"]
    ne, ni = len(xe), len(xi)

    def assembly_rate(rows_e, rows_i, grow):
        while True:
            re_ = rng.choice(ne, rows_e, replace=False)
            ri_ = rng.choice(ni, rows_i, replace=False)
            t0 = time.perf_counter()
            O.assemble(xe, te, c["k_ext"], rows=re_)
            Oi = O.assemble(xi, ti, c["k_int"], rows=ri_)
            dt = time.perf_counter() - t0
            if not grow or dt > budget_s / 4 or rows_e > 4000:
                return rows_e, rows_i, dt, ri_, Oi
            scale = max(2.0, min(8.0, budget_s / max(dt, 1e-3) / 2))
            rows_e, rows_i = int(rows_e * scale), int(rows_i * scale)

    rows_e, rows_i, dt, ri_, Oi = assembly_rate(8, 6, True)
    entries = 4 * (rows_e * ne + rows_i * ni)
    O.set_threads(1)
    r1e, r1i, dt1, _, _ = assembly_rate(max(2, rows_e // (2 * threads)), max(2, rows_i // (2 * threads)), False)
    O.set_threads(threads)
    ent1 = 4 * (r1e * ne + r1i * ni)
    # oracle mat-vec on 2 x rows_i rows of the printed matrix
    P = O.mortar(c["int"], c["ext"], rows=ri_)
    rr = c["rho_int"] / c["rho_ext"]
    n = 2 * ne + 2 * ni
    A = np.zeros((2 * len(ri_), n), dtype=np.complex128)
    A[:len(ri_), :ne] = -0.5 * P
    A[:len(ri_), 2 * ne:2 * ne + ni] = -Oi["K"]
    A[:len(ri_), 2 * ne + ni:] = Oi["V"]
    A[len(ri_):, ne:2 * ne] = -0.5 * rr * P
    A[len(ri_):, 2 * ne:2 * ne + ni] = Oi["D"]
    A[len(ri_):, 2 * ne + ni:] = Oi["T"]
    # repeat the sampled rows to at least 1024 (about 600 MB), so that the
    # product streams from memory as the full one does
    A = np.resize(A, (max(1024, A.shape[0]), n))
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    A @ x
    reps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < 2.0:
        A @ x
        reps += 1
    dmv = (time.perf_counter() - t0) / reps
    out = {"value": round(entries / dt / 1e9, 6), "unit": "Gentries/s", "cores": threads, "kind": "oracle",
           "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
           "sample": f"oracle V/K/T/D rows: {rows_e} of {ne} exterior + {rows_i} of {ni} interior "
                     f"({entries} entries, {dt:.1f} s, {threads} threads)",
           "one_thread": {"value": round(ent1 / dt1 / 1e9, 6), "unit": "Gentries/s",
                          "sample": f"{r1e} + {r1i} rows ({ent1} entries, {dt1:.1f} s)"},
           "matvec": {"GBps": round(16.0 * A.size / dmv / 1e9, 2), "rows": int(A.shape[0]), "cols": n,
                      "ms": round(1e3 * dmv, 3),
                      "full_matvec_ms_at_this_rate": round(1e3 * dmv * n / A.shape[0], 1)}}
    meta = os.path.join(ROOT, "tests", "golden", f"mtf_{c['name']}.json")
    if os.path.exists(meta):
        with open(meta) as f:
            m = _json.load(f)
        out["solve_recorded"] = {"wall_s": m["wall_s"], "threads": m["threads"],
                                 "what": "oracle assembly of every row, dense mortar, LU of the full system "
                                         "(tests/golden/make_mtf_traces.py), on the build container's host, "
                                         "not the GPU box"}
    return out


def run_workload(ctx, B, c, prec, tol, steps, warmup, timed=(), breakdown=()):
    """`warmup` untimed and `steps` timed passes of the whole path on
    workload c: mesh tables, problem, operators, projection, solve; traces
    left in device memory.  Returns per-step phases and latencies, the
    kernel times of `timed` over the timed steps, the last traces and, with
    `breakdown`, the times of those kernels over one further step."""
    import torch
    (xe, te), (xi, ti) = c["ext"], c["int"]

    def step(ph):
        t = time.perf_counter()
        me, mi = B.Mesh(ctx, xe, te), B.Mesh(ctx, xi, ti)
        p = B.Problem(ctx, me, mi, c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"], precision=prec)
        t1 = time.perf_counter()
        p.assemble_operators()
        t2 = time.perf_counter()
        p.assemble_projection()
        t3 = time.perf_counter()
        out, stats, code = p.solve(c["dirs"], tol=tol, maxit=3000)
        torch.cuda.synchronize()   # traces stay in device memory (HBM-resident output)
        t4 = time.perf_counter()
        for k, v in (("mesh_problem", t1 - t), ("operators_enqueue", t2 - t1), ("projection", t3 - t2),
                     ("solve", t4 - t3), ("assembly_device", 1e-3 * stats["t_assembly_ms"])):
            ph.setdefault(k, []).append(v)
        assert code == B.OK, stats
        return out, stats

    for _ in range(warmup):
        step({})
    torch.cuda.synchronize()
    ctx.set_kernel_timing(timed)
    phases, lat, iters = {}, [], []
    t_start = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        x, stats = step(phases)
        lat.append(time.perf_counter() - t0)
        iters.append(stats["iterations"])
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    ktimes = {k: ctx.kernel_time(k) for k in timed}
    ctx.set_kernel_timing(())
    out = dict(total=total, lat=lat, phases=phases, iters=iters, stats=stats, x=x.cpu().numpy()[0], ktimes=ktimes)
    if breakdown:
        # every kernel's events cost a few microseconds of issue each, so the
        # per-kernel breakdown comes from one more step after the timed ones
        ctx.set_kernel_timing(breakdown)
        step({})
        torch.cuda.synchronize()
        out["breakdown"] = {k: ctx.kernel_time(k) for k in breakdown}
        ctx.set_kernel_timing(())
    return out


def summarise(c, r, steps, prec, tol, name):
    """The per-workload figures of one run_workload result."""
    import numpy as np
    ne, ni = len(c["ext"][0]), len(c["int"][0])
    entries = 4 * ne * ne + 4 * ni * ni
    med = {k: round(1e3 * statistics.median(v), 3) for k, v in r["phases"].items()}
    ref = golden(name)
    return {"workload": workload_name(c, prec, tol),
            "gentries_per_s": round(entries * steps / r["total"] / 1e9, 4),
            "ms_per_step": round(1e3 * r["total"] / steps, 3),
            "assembly_gentries_per_s": round(entries / (med["assembly_device"] * 1e-3) / 1e9, 3),
            "solves_per_s": round(steps / r["total"], 3),
            "p50_ms": round(1e3 * statistics.median(r["lat"]), 3),
            "p99_ms": round(1e3 * float(np.percentile(r["lat"], 99)), 3),
            "phase_ms": med,
            "gmres_iterations": int(statistics.median(r["iters"])),
            "ir_steps": r["stats"]["ir_steps"],
            "rel_residual": r["stats"]["rel_residual"],
            "trace_rel_err_vs_oracle": None if ref is None else trace_error(r["x"], ref[0], ne, ni)}


def workload_name(c, prec, tol):
    body = "sphere" if tuple(c["axes"]) == (1.0, 1.0, 1.0) else "ellipsoid"
    ne, ni = len(c["ext"][0]), len(c["int"][0])
    form = "FP64" if prec == 0 else "mixed (complex64 operators, FP64 Arnoldi and refinement)"
    return (f"{body}-ico{c['ext_level']}/fib{ni} MTF, {form}, n_ext {ne}, n_int {ni}, "
            f"k {c['k_ext']:g}/{c['k_int']:g}, rho ratio {c['rho_int'] / c['rho_ext']:g}, 1 plane wave, "
            f"GMRES tol {tol:g}")


def precision_compare(ctx, B, synth, np, fp64, steps=2, tol=1e-7):
    """The mixed form (complex64 operators, FP32-accumulated products, FP64
    Arnoldi and refinement residuals) on the headline workload, end to end,
    against the FP64 headline run: step time, solves/s, iterations, the
    mat-vec bandwidth, and the trace errors of both forms against the
    oracle's exact discrete solution and against each other."""
    c = synth.make_config("C3")
    ne, ni = len(c["ext"][0]), len(c["int"][0])
    r = run_workload(ctx, B, c, B.C64_MIXED, tol, steps, 1, ("mtf_dense",))
    ms, n = r["ktimes"]["mtf_dense"]
    res = summarise(c, r, steps, B.C64_MIXED, tol, "C3")
    res["mtf_dense_us"] = round(1e3 * ms / n, 2)
    res["mtf_dense_GBps"] = round(8 * (ne * ne + ne * (ne + 1) + ni * ni + ni * (ni + 1)) / (ms / n * 1e-3) / 1e9, 1)
    res["trace_rel_err_mixed_vs_fp64"] = trace_error(r["x"], fp64["x"], ne, ni)
    res["speedup_mixed_vs_fp64"] = round(steps / r["total"] / fp64["solves_per_s"], 3)
    return res


FP32_MFMA_TFLOPS = 157.3    # MI355X dense FP32 matrix-core peak, TFLOP/s


def batching_compare(ctx, B, synth, np, tol=1e-7, sample=2):
    """The batching workload (ellipsoid (1, 0.8, 0.6), ico L5 with 10242 nodes
    / Fibonacci 8000 nodes, k 8 / 12, rho ratio 2, 64 plane waves): one block
    solve of all 64 directions in the mixed form (64 independent GMRES runs
    sharing one matrix-core product per step) against one-at-a-time solves of
    the mixed and of the plain FP64 form, timed on the first `sample`
    directions.  tol 1e-7 for all forms (the tolerance at which the traces of
    every form lie within 1e-5 of the exact discrete solution).  The block
    GEMM is reported against the FP32 matrix-core peak with 2048 (N_e^2 +
    N_i^2) useful flops per launch (8 real flops per complex multiply-add, 4
    blocks per mesh, 64 vectors)."""
    import torch
    c = synth.make_config("C4")
    (xe, te), (xi, ti) = c["ext"], c["int"]
    ne, ni = len(xe), len(xi)
    dirs = c["dirs"]

    def setup(prec):
        me, mi = B.Mesh(ctx, xe, te), B.Mesh(ctx, xi, ti)
        p = B.Problem(ctx, me, mi, c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"], precision=prec)
        p.assemble_operators()
        p.assemble_projection()
        return p, me, mi

    res = {}
    p, me, mi = setup(B.C64_MIXED)
    p.solve(dirs, tol=1e-2, maxit=20, batch=64)   # first use of the class: the tuner times the GEMM shapes
    torch.cuda.synchronize()
    ctx.set_kernel_timing(("block_gemm", "mass_gemm", "mass_apply"))
    t0 = time.perf_counter()
    out, st, code = p.solve(dirs, tol=tol, maxit=1500, batch=64)
    blk = out.cpu().numpy()
    dt = time.perf_counter() - t0
    assert code == B.OK, st
    gms, gn = ctx.kernel_time("block_gemm")
    mms, mn = ctx.kernel_time("mass_gemm")
    ams, an = ctx.kernel_time("mass_apply")
    ctx.set_kernel_timing(())
    flops = 2048.0 * (ne * ne + ni * ni)
    ach = flops / (gms / gn * 1e-3) / 1e12
    res["block_c64_mixed"] = {"solves": 64, "solve_ms": round(1e3 * dt, 1), "solves_per_s": round(64 / dt, 2),
                              "iterations_total": st["iterations"], "ir_steps": st["ir_steps"],
                              "rel_residual": st["rel_residual"]}
    res["roofline"] = {"kernel": "block_gemm", "bound": "mfma", "achieved": round(ach, 1), "peak": FP32_MFMA_TFLOPS,
                       "unit": "TFLOP/s", "frac": round(ach / FP32_MFMA_TFLOPS, 4), "traffic": None,
                       "avg_launch_us": round(1e3 * gms / gn, 1), "flop_per_launch": flops,
                       "inverse_mass": ({"form": "dense on the matrix cores",
                                         "tflops": round(512.0 * (ne * ne + ni * ni) / (mms / mn * 1e-3) / 1e12, 1)}
                                        if mn else {"form": "sparse Chebyshev", "ms_per_step": round(
                                            ams / max(1, an) * 3, 3)})}
    t0 = time.perf_counter()
    seq, s1, c1 = p.solve(dirs[:sample], tol=tol, maxit=1500)
    seq = seq.cpu().numpy()
    dt1 = time.perf_counter() - t0
    res["single_c64_mixed"] = {"solves": sample, "ms_per_solve": round(1e3 * dt1 / sample, 1),
                               "solves_per_s": round(sample / dt1, 2), "iterations": s1["iterations"]}
    del p, me, mi
    p, me, mi = setup(B.C128)
    t0 = time.perf_counter()
    ref, s2, c2 = p.solve(dirs[:sample], tol=tol, maxit=1500)
    ref = ref.cpu().numpy()
    dt2 = time.perf_counter() - t0
    res["single_fp64"] = {"solves": sample, "ms_per_solve": round(1e3 * dt2 / sample, 1),
                          "solves_per_s": round(sample / dt2, 2), "iterations": s2["iterations"]}
    del p, me, mi
    err = max(trace_error(blk[r], ref[r], ne, ni) for r in range(sample))
    gold = golden("C4")
    if gold is not None:
        res["block_c64_mixed"]["trace_rel_err_vs_oracle"] = max(trace_error(blk[r], gold[r], ne, ni)
                                                                for r in range(len(dirs)))
        res["single_c64_mixed"]["trace_rel_err_vs_oracle"] = max(trace_error(seq[r], gold[r], ne, ni)
                                                                 for r in range(sample))
        res["single_fp64"]["trace_rel_err_vs_oracle"] = max(trace_error(ref[r], gold[r], ne, ni)
                                                            for r in range(sample))
    res["tuned_shapes"] = {k: v for k, v in B.tune_table().items() if k.startswith("gemm-ops:c128")}
    return {"workload": f"ellipsoid-ico5/fib8000 MTF (n_ext {ne}, n_int {ni}, k 8/12, rho ratio 2), 64 plane waves, "
                        f"GMRES tol {tol:g}",
            **res, "trace_rel_err_block_vs_fp64": err,
            "speedup_block_vs_fp64": round(res["block_c64_mixed"]["solves_per_s"] / res["single_fp64"]["solves_per_s"],
                                           2),
            "speedup_block_vs_single_mixed": round(res["block_c64_mixed"]["solves_per_s"] /
                                                   res["single_c64_mixed"]["solves_per_s"], 2)}


def serving_run(B, synth, n_requests=24, n_sustained=32, slots=4, tol=1e-5, maxit=1000):
    """The serving workload: the seeded Poisson stream (random ellipsoids with
    semi-axes in [0.5, 1.5], exterior icosphere L3-L5, interior Fibonacci grid
    at 0.7-1.3 times the exterior node count, k_ext in [1, 15], k_int = k_ext
    x [1.2, 2.5], rho ratio 1.5, 1-16 plane waves) through a server with
    `slots` workers (mixed precision, all directions of a request solved
    together, admission by device footprint with bounded out-of-order entry).
    Two runs: the first `n_requests` released at the stream's own rate (mean
    20 per second, far above what one device completes, so latency is
    mostly queueing), and the first `n_sustained` at 70 % of the request rate
    the first run completed (arrival times of the same stream, scaled), where
    latency is mostly service.  solves/s counts only directions of requests
    that converged.  Meshes are generated before the clock starts (they are
    the requests' inputs)."""
    from paper_2206_00708_amd import serve
    qs = synth.serving_stream()[:max(n_requests, n_sustained)]
    reqs = []
    for i, q in enumerate(qs):
        ext, inte = synth.request_meshes(q)
        reqs.append(serve.Request(i, q["t_arrival"], ext, inte, q["k_ext"], q["k_int"], q["rho_ext"], q["rho_int"],
                                  synth.request_directions(q)))

    def run(rs):
        srv = serve.Server(slots=slots, tol=tol, maxit=maxit)
        res, summ = srv.run(rs, realtime=True)
        srv.close()
        iters = [r.stats["iterations"] for r in res.values() if r.stats]
        summ["iterations_median"] = int(statistics.median(iters)) if iters else 0
        return summ

    out = {"workload": f"seeded Poisson stream of random ellipsoids, ext L3-L5, complex64 + FP64 refinement, "
                       f"tol {tol:g}, maxit {maxit}, {slots} workers"}
    s1 = run(reqs[:n_requests])
    s1["offered_req_per_s"] = 20.0
    out["stated_rate"] = s1
    cap = max(s1["completed"] / s1["makespan_s"], 1e-3)
    scale = n_sustained / (0.7 * cap * qs[n_sustained - 1]["t_arrival"])   # stretch of the arrival times
    rs = [serve.Request(r.id, r.t_arrival * scale, r.ext, r.inte, r.k_ext, r.k_int, r.rho_ext, r.rho_int, r.dirs)
          for r in reqs[:n_sustained]]
    s2 = run(rs)
    s2["offered_req_per_s"] = round(n_sustained / (qs[n_sustained - 1]["t_arrival"] * scale), 3)
    out["sustained"] = s2
    return out


# FP64 operations per quadrature-point evaluation of the field kernel (FMA =
# 2): y - x 3, r^2 5, 1/r 1, k r 2, phase reduction and sin/cos polynomials
# 45, exp(ikr)/r 2, (y - x).n / r^2 7, the radial factor 6, the two complex
# products and sums 16.
FIELD_FLOP_PER_EVAL = 87


def field_run(ctx, B, synth, np, reps=5):
    """Field evaluation on the C2 body: the traces of one solve, then the
    total field on a 100 x 100 grid of the plane z = 0 over [-2, 2]^2 (the
    paper's accuracy grid, 100 x 100 points over the body and a margin of
    half its size, Sec. 5.3), regions from the exterior mesh's winding
    number.  Reports the field call's wall time, the field kernel's device
    time (HIP events) and its FP64 rate by the operation count above."""
    import torch
    c = synth.make_config("C2")
    me, mi = B.Mesh(ctx, *c["ext"]), B.Mesh(ctx, *c["int"])
    p = B.Problem(ctx, me, mi, c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"])
    p.assemble_operators()
    p.assemble_projection()
    x, st, code = p.solve(c["dirs"], tol=c["tol"], maxit=2000)
    g = np.linspace(-2.0, 2.0, 100)
    gx, gy = np.meshgrid(g, g, indexing="ij")
    pts = torch.as_tensor(np.stack([gx.ravel(), gy.ravel(), np.zeros(gx.size)], axis=1), device=ctx.device)
    (me.winding(pts) > 0.5).to(torch.int32)   # warm-up (first launches load the kernels, torch's too)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    region = (me.winding(pts) > 0.5).to(torch.int32)
    torch.cuda.synchronize()
    t_wind = time.perf_counter() - t0
    p.field(c["dirs"], x, pts, region)   # warm-up
    ctx.set_kernel_timing(("field",))
    lat = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        f = p.field(c["dirs"], x, pts, region)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0)
    ms, n = ctx.kernel_time("field")
    ctx.set_kernel_timing(())
    n_in = int(region.sum().item())
    n_out = pts.shape[0] - n_in
    evals = 6 * (n_out * len(c["ext"][1]) + n_in * len(c["int"][1]))
    dev_ms = ms / reps   # both regions' launches of one call
    tf = FIELD_FLOP_PER_EVAL * evals / (dev_ms * 1e-3) / 1e12
    return {"workload": "C2 body, 100 x 100 grid on z = 0 over [-2, 2]^2, 1 plane wave",
            "points": int(pts.shape[0]), "interior_points": n_in, "quadrature_evaluations": evals,
            "call_ms": round(1e3 * float(np.median(lat)), 3), "kernel_ms": round(dev_ms, 3),
            "points_per_s": round(pts.shape[0] / float(np.median(lat)), 1),
            "winding_ms": round(1e3 * t_wind, 3),
            "roofline": {"kernel": "field_partial", "bound": "alu", "achieved": round(tf, 2), "peak": 78.6,
                         "unit": "TFLOP/s", "frac": round(tf / 78.6, 4), "flop_per_eval": FIELD_FLOP_PER_EVAL},
            "max_abs_field": round(float(f.abs().max().item()), 4)}


def pmchwt_run(ctx, B, synth, np, reps=3):
    """The exterior PMCHWT and high-contrast Neumann formulations (Sec. 3.3)
    beside the multiple-traces one on the C2 workload, after the same
    assembly: GMRES iterations, solve time, time per iteration, and the
    relative difference of the exterior traces (PMCHWT unknowns p and
    dp/dn+, high-contrast dp/dn+ and mu, multiple-traces -v_ext and -w_ext;
    all solved to the workload's tolerance, 1e-6)."""
    import torch
    c = synth.make_config("C2")
    me, mi = B.Mesh(ctx, *c["ext"]), B.Mesh(ctx, *c["int"])
    p = B.Problem(ctx, me, mi, c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"])
    p.assemble_operators()
    p.assemble_projection()
    p.solve_pmchwt(c["dirs"], tol=c["tol"], maxit=2000)   # warm-up
    res = {}
    p.solve_hc_neumann(c["dirs"], tol=c["tol"], maxit=2000)   # warm-up
    for name in ("pmchwt", "hc_neumann", "mtf"):
        lat = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "pmchwt":
                x, st, code = p.solve_pmchwt(c["dirs"], tol=c["tol"], maxit=2000)
            elif name == "hc_neumann":
                x, st, code = p.solve_hc_neumann(c["dirs"], tol=c["tol"], maxit=2000)
            else:
                x, st, code = p.solve(c["dirs"], tol=c["tol"], maxit=2000)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0)
        t = float(np.median(lat))
        res[name] = {"iterations": st["iterations"], "solve_ms": round(1e3 * t, 3),
                     "ms_per_iteration": round(1e3 * t / max(1, st["iterations"]), 4),
                     "rel_residual": st["rel_residual"], "code": int(code)}
        res[name + "_x"] = x.cpu().numpy()[0]
    ne = len(c["ext"][0])
    a, h, b = res.pop("pmchwt_x"), res.pop("hc_neumann_x"), res.pop("mtf_x")
    e = lambda u, v: float(np.linalg.norm(u - v) / np.linalg.norm(v))
    res["trace_rel_diff_p"] = e(a[:ne], -b[:ne])
    res["trace_rel_diff_dpdn"] = e(a[ne:], -b[ne:2 * ne])
    res["hc_neumann_rel_diff_dpdn"] = e(h[:ne], -b[ne:2 * ne])
    res["workload"] = "C2 (sphere ico4 / Fibonacci 2002, k 5/8, rho ratio 1.5), 1 plane wave, tol 1e-6"
    return res


def mortar_run(ctx, B, synth, np):
    """The mortar step of the projection set-up (Sec. 3.1) with its geometry
    on the host threads and on the device, at C3 (ellipsoid ico5 / Fibonacci
    8002) and on a sphere pair with a denser interior grid (ico5, 10242 nodes /
    Fibonacci 16000; the dense inverse masses take at most 16384 nodes):
    wall time of the step (geometry and CSR), the device kernels' time, and
    whether the two give the same matrix."""
    import torch
    cases = [("C3", synth.make_config("C3")),
             ("sphere ico5 / Fibonacci 16000", None)]
    res = {}
    for name, c in cases:
        if c is None:
            ext, inte, _ = synth.configs.make_pair(13, 5, "fib", 0.01, (1.0, 1.0, 1.0), int_n=16000)
            c = {"ext": ext, "int": inte, "k_ext": 5.0, "k_int": 8.0}
        me, mi = B.Mesh(ctx, *c["ext"]), B.Mesh(ctx, *c["int"])
        out = {"n_ext": len(c["ext"][0]), "n_int": len(c["int"][0])}
        P = {}
        for on in (False, True, False, True):   # each setting twice; the second run is reported
            p = B.Problem(ctx, me, mi, c["k_ext"], c["k_int"], 1.0, 1.5)
            p.set_mortar(on)
            if on:
                ctx.set_kernel_timing(("mortar",))
            p.assemble_projection()
            key = "device" if on else "host"
            out[key + "_ms"] = round(p.mortar_ms(), 3)
            if on:
                out["device_kernel_ms"] = round(ctx.kernel_time("mortar")[0], 3)
                ctx.set_kernel_timing(())
            P[key] = p.projection()
            del p
            torch.cuda.synchronize()
        (rh, ch, vh), (rd, cd, vd) = P["host"], P["device"]
        out["nnz"] = int(len(vh))
        out["same_sparsity"] = bool(np.array_equal(rh, rd) and np.array_equal(ch, cd))
        out["max_rel_value_diff"] = float(np.abs(vh - vd).max() / np.abs(vh).max()) if out["same_sparsity"] else None
        out["speedup"] = round(out["host_ms"] / out["device_ms"], 2)
        res[name] = out
    return res


def incident_run(ctx, B, synth, np):
    """The C2 workload with the foam model's variations (Sec. 5.7) beside the
    lossless plane wave: an absorbing interior (k_int + 0.5 i, the
    complex-wavenumber instantiation of the regular assembly) and a point
    source at (0, 0, 3): regular-assembly kernel time, GMRES steps and solve
    time to the workload tolerance."""
    import torch
    c = synth.make_config("C2")
    res = {}
    for name, kim, kind, src in (("plane wave", 0.0, 0, c["dirs"]),
                                 ("absorbing interior, k_int + 0.5i", 0.5, 0, c["dirs"]),
                                 ("point source at (0, 0, 3)", 0.0, 1, np.array([[0.0, 0.0, 3.0]]))):
        me, mi = B.Mesh(ctx, *c["ext"]), B.Mesh(ctx, *c["int"])
        p = B.Problem(ctx, me, mi, c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"])
        p.set_k_int_imag(kim)
        p.set_incident(kind)
        ctx.set_kernel_timing(("regular_tiles",))
        p.assemble_operators()
        p.assemble_projection()
        reg_ms = ctx.kernel_time("regular_tiles")[0]
        ctx.set_kernel_timing(())
        p.solve(src, tol=c["tol"], maxit=2000)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, st, code = p.solve(src, tol=c["tol"], maxit=2000)
        torch.cuda.synchronize()
        res[name] = {"regular_kernel_ms": round(reg_ms, 3), "iterations": st["iterations"],
                     "solve_ms": round(1e3 * (time.perf_counter() - t0), 3), "rel_residual": st["rel_residual"],
                     "code": int(code)}
        del p, me, mi
    res["workload"] = "C2 (sphere ico4 / Fibonacci 2002, k 5/8, rho ratio 1.5), tol 1e-6"
    return res


def progress(what, t0):
    """One line on stderr per finished section (stdout carries only the JSON line)."""
    print(f"bench: {what} done ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=("C3", "C2"), default="C3",
                    help="headline workload: C3 (ellipsoid ico5/fib8002, the default) or C2 (sphere ico4/fib2002), "
                         "both FP64")
    ap.add_argument("--no-c2", action="store_true", help="skip the C2 sub-object")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true", help="skip the FP64 vs mixed comparison")
    ap.add_argument("--no-batching", action="store_true", help="skip the multi-RHS comparison")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream")
    ap.add_argument("--no-field", action="store_true", help="skip the field evaluation")
    ap.add_argument("--no-pmchwt", action="store_true", help="skip the comparison of the exterior formulations")
    ap.add_argument("--no-mortar", action="store_true", help="skip the host vs device mortar comparison")
    ap.add_argument("--no-incident", action="store_true", help="skip the absorbing-interior and point-source runs")
    ap.add_argument("--headline-only", action="store_true", help="skip every section after the headline")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes 5 times (reference for the "
                         "HBM byte counters) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "multi-GPU sharding of the operators is a design note, not implemented", file=sys.stderr)
        sys.exit(2)
    if args.headline_only:
        for k in ("c2", "cpu_baseline", "precision", "batching", "serving", "field", "pmchwt", "mortar", "incident"):
            setattr(args, "no_" + k.replace("-", "_"), True)

    import numpy as np
    import torch

    import paper_2206_00708_amd as B
    import synth

    name = args.workload
    tol = HEADLINE_TOL[name]
    c = synth.make_config(name)
    (xe, te), (xi, ti) = c["ext"], c["int"]
    ne, ni = len(xe), len(xi)
    entries = 4 * ne * ne + 4 * ni * ni
    torch.cuda.init()
    ctx = B.Context(0)
    # the timed steps carry events on the two roofline kernels only
    timed = ("regular_tiles", "mtf_dense")
    breakdown = ("regular_tiles", "gather_tiles", "singular_pairs", "mtf_dense", "mass_apply", "cgs_dots",
                 "cgs_update", "arnoldi_finish", "krylov_normalize")
    t_bench = time.perf_counter()
    r = run_workload(ctx, B, c, B.C128, tol, args.steps, args.warmup, timed, breakdown)
    head = summarise(c, r, args.steps, B.C128, tol, name)
    progress("headline " + name, t_bench)
    ktimes = r["ktimes"]
    # algorithmic work per launch
    # K in full and the upper triangles of V and D (T = K^T), complex128, both meshes
    mv_bytes = 16.0 * (ne * ne + ne * (ne + 1) + ni * ni + ni * (ni + 1))
    pairs = 0.5 * (len(te) ** 2 + len(ti) ** 2)                    # unordered triangle pairs per step
    reg_flops = pairs * 36 * FLOP_PER_POINT_PAIR
    ms, n = ktimes["mtf_dense"]
    ach = mv_bytes / (ms / n * 1e-3) / 1e9
    # the GMRES steps inside captured graphs carry no events: the timed launches are the steps issued one
    # by one (the first batch and the last steps of each solve) and the residual products; the kernel's
    # time per step is its average launch times its launches per step (one per Arnoldi step plus the
    # final residual and the completing step)
    mv_launches = head["gmres_iterations"] + 2
    roof_mv = {"kernel": "mtf_sym_tile", "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
               "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": counted_traffic("mtf_dense", name),
               "avg_launch_us": round(1e3 * ms / n, 2), "bytes_per_launch": mv_bytes,
               "timed_launches_per_step": round(n / args.steps, 1), "launches_per_step": mv_launches,
               "ms_per_step": round(ms / n * mv_launches, 3)}
    ms, n = ktimes["regular_tiles"]
    ach = reg_flops / (ms / args.steps * 1e-3) / 1e12
    roof_reg = {"kernel": "regular_tiles", "bound": "alu", "achieved": round(ach, 2), "peak": FP64_VEC_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / FP64_VEC_TFLOPS, 4), "traffic": None,
                "avg_launch_us": round(1e3 * ms / n, 2), "flop_per_step_model": reg_flops,
                "ms_per_step": round(ms / args.steps, 3), "counters": counted_valu("regular_tiles", name, ms / n)}
    dominant = max((roof_mv, roof_reg), key=lambda r: r["ms_per_step"])
    roof, roof_other = (roof_mv, roof_reg) if dominant is roof_mv else (roof_reg, roof_mv)
    line = {
        "metric": "dense BEM assembly Gentries/s; solves/s vs plain FP64 at 1e-5 err; p99 latency",
        "value": round(entries * args.steps / r["total"] / 1e9, 4),
        "unit": "Gentries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * r["total"] / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": head["workload"], "n_ext": ne, "n_int": ni, "k_ext": c["k_ext"], "k_int": c["k_int"],
                   "rho_ratio": c["rho_int"] / c["rho_ext"], "gmres_tol": tol},
        "roofline": roof,
        "roofline_other": roof_other,
        **{k: v for k, v in head.items() if k not in ("workload", "gentries_per_s", "ms_per_step")},
        "kernel_ms_per_step": {k: round(v[0], 3) for k, v in r["breakdown"].items()},
        "kernel_launches_per_step": {k: v[1] for k, v in r["breakdown"].items()},
        "kernel_breakdown_note": "one untimed step after the timed ones, with events on every listed kernel; the "
                                 "GMRES steps inside captured graphs carry no events, so the Krylov-step kernels "
                                 "count only the steps issued one by one",
        "tuned_shapes": {k: v for k, v in B.tune_table().items() if k.startswith("mtf-")},
    }
    if not args.no_c2 and name != "C2":
        c2 = synth.make_config("C2")
        line["c2"] = summarise(c2, run_workload(ctx, B, c2, B.C128, c2["tol"], args.steps, args.warmup), args.steps,
                               B.C128, c2["tol"], "C2")
        progress("c2", t_bench)
    if not args.no_precision:
        line["precision"] = precision_compare(ctx, B, synth, np, {"x": r["x"], "solves_per_s": head["solves_per_s"]})
        progress("precision", t_bench)
    ctx.trim()
    if not args.no_batching:
        line["batching"] = batching_compare(ctx, B, synth, np)
        progress("batching", t_bench)
    if not args.no_field:
        line["field"] = field_run(ctx, B, synth, np)
        progress("field", t_bench)
    if not args.no_pmchwt:
        line["pmchwt"] = pmchwt_run(ctx, B, synth, np)
        progress("pmchwt", t_bench)
    if not args.no_mortar:
        line["mortar"] = mortar_run(ctx, B, synth, np)
        progress("mortar", t_bench)
    if not args.no_incident:
        line["incident"] = incident_run(ctx, B, synth, np)
        progress("incident", t_bench)
    if not args.no_serving:
        ctx.trim()   # the serving workers size their budget from free HBM: return this context's blocks first
        torch.cuda.empty_cache()
        line["serving"] = serving_run(B, synth)
        progress("serving", t_bench)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_oracle_baseline(c)
        progress("cpu_baseline", t_bench)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
