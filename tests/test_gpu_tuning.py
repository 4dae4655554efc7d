"""The kernel-shape tuner: the first block solve of a size class times the
GEMM's K splits (per mesh) and stage depth and the first solve the mat-vec's tile edge,
records them in the process-wide table (and its file), and later problems of
the class reuse them, so that their results are bitwise equal."""
import os

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2206_00708_amd")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a device"
    return B.Context(0)


def _problem(ctx, c, prec):
    me, mi = B.Mesh(ctx, *c["ext"]), B.Mesh(ctx, *c["int"])
    p = B.Problem(ctx, me, mi, c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"], precision=prec)
    p.assemble_operators()
    p.assemble_projection()
    return p, me, mi


def test_shapes_recorded_and_reused(ctx):
    c = synth.make_config("C1")
    dirs = synth.plane_wave_directions(4, np.random.default_rng(3))
    p, me, mi = _problem(ctx, c, B.C64_MIXED)
    x1, s1, code = p.solve(dirs, tol=1e-8, maxit=500, batch=4)
    assert code == B.OK
    t1 = B.tune_table()
    gemm = [k for k in t1 if k.startswith("gemm-ops:")]
    mtf = [k for k in t1 if k.startswith("mtf-c64:")]
    print("tuning table:", t1)
    assert gemm and mtf
    for k in gemm:   # K chunks of the exterior and interior segments, k per LDS stage
        nke, nki, kst = t1[k]
        assert 1 <= nke <= 8 and 1 <= nki <= 8 and kst in (32, 64)
    for k in mtf:
        assert t1[k][0] in (64, 128)
    # a second problem of the same class: the recorded shapes, the same bits
    q, me2, mi2 = _problem(ctx, c, B.C64_MIXED)
    x2, s2, code2 = q.solve(dirs, tol=1e-8, maxit=500, batch=4)
    assert code2 == B.OK
    assert B.tune_table() == t1
    assert torch.equal(x1, x2)
    # the file holds the same entries
    path = os.environ.get("BEMTX_TUNE_FILE") or os.path.join(
        os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache"), "bemtx",
        "tune-gfx950.txt")
    if os.path.exists(path):
        with open(path) as f:
            text = f.read()
        assert all(k in text for k in gemm + mtf)


def test_fp64_tile_edge(ctx):
    c = synth.make_config("C1")
    p, me, mi = _problem(ctx, c, B.C128)
    out, st, code = p.solve(c["dirs"], tol=1e-8, maxit=500)
    assert code == B.OK
    assert any(k.startswith("mtf-c128:") for k in B.tune_table())


def test_old_format_entry_tuned_again(tmp_path):
    """A table file holding the operator GEMM's entry in the older two-value
    form (one K split for both meshes): the first block solve of that class
    times the shapes again and replaces the entry with the three-value form.
    Run in a child process, since the table is read once per process."""
    import math
    import subprocess
    import sys
    c = synth.make_config("C1")
    cls = lambda n: round(4 * math.log2(n))
    key = f"gemm-ops:c32:e{cls(len(c['ext'][0]))}:i{cls(len(c['int'][0]))}"   # 4 runs: 8 real columns, 32-wide tile
    f = tmp_path / "tune.txt"
    f.write_text(f"{key} 4 32\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import sys, numpy as np; sys.path.insert(0, %r); sys.path.insert(0, %r)\n"
        "import synth, paper_2206_00708_amd as B\n"
        "c = synth.make_config('C1'); ctx = B.Context(0)\n"
        "me, mi = B.Mesh(ctx, *c['ext']), B.Mesh(ctx, *c['int'])\n"
        "p = B.Problem(ctx, me, mi, c['k_ext'], c['k_int'], c['rho_ext'], c['rho_int'], precision=B.C64_MIXED)\n"
        "p.assemble_operators(); p.assemble_projection()\n"
        "x, s, code = p.solve(synth.plane_wave_directions(4, np.random.default_rng(3)), tol=1e-8, maxit=500, batch=4)\n"
        "assert code == B.OK\n"
        "print(B.tune_table()[%r])\n" % (root, os.path.join(root, "tests"), key))
    env = dict(os.environ, BEMTX_TUNE_FILE=str(f))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=240, env=env)
    assert out.returncode == 0, out.stderr[-2000:]
    v = eval(out.stdout.strip().splitlines()[-1])
    print("re-tuned entry:", key, v)
    assert len(v) == 3 and 1 <= v[0] <= 8 and 1 <= v[1] <= 8 and v[2] in (32, 64)
    assert f"{key} {v[0]} {v[1]} {v[2]}" in f.read_text()
