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
