"""GMRES steps in captured HIP graphs against the same steps launched one by
one (bem_problem_set_graphs), through the C ABI.  The kernels, their order
and arithmetic are the same in both modes, so the traces, iteration counts
and residuals must agree bit for bit: single FP64 runs (C1; C2 with more than
one 64-step graph range), the mixed single run, the matrix-core block of
several directions, the exterior PMCHWT system, a context on a torch side
stream, and replays across consecutive solves with other device work and
synchronisations between them (every replay checked against the launches
one by one)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2206_00708_amd")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a device"
    c = B.Context(0)
    yield c
    c.trim()


def _problem(ctx, c, prec):
    me, mi = B.Mesh(ctx, *c["ext"]), B.Mesh(ctx, *c["int"])
    p = B.Problem(ctx, me, mi, c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"], precision=prec)
    p.assemble_operators()
    p.assemble_projection()
    return p, me, mi


def _both(p, dirs, **kw):
    p.set_graphs(False)
    xe, se, ce = p.solve(dirs, **kw)
    p.set_graphs(True)
    xg, sg, cg = p.solve(dirs, **kw)
    return (xe.cpu().numpy(), se, ce), (xg.cpu().numpy(), sg, cg)


def _same(a, b, tag):
    (xe, se, ce), (xg, sg, cg) = a, b
    print(f"{tag}: {se['iterations']} steps, {sg['graph_steps']} in graphs, residual {sg['rel_residual']:.2e}")
    assert ce == cg == B.OK, (se, sg)
    assert se["graph_steps"] == 0
    assert sg["graph_steps"] > 0
    assert se["iterations"] == sg["iterations"] and se["ir_steps"] == sg["ir_steps"]
    assert se["rel_residual"] == sg["rel_residual"]
    assert np.array_equal(xe, xg), float(np.abs(xe - xg).max())


def test_fp64_c1(ctx):
    c = synth.make_config("C1")
    p, me, mi = _problem(ctx, c, B.C128)
    _same(*_both(p, c["dirs"], tol=1e-12, maxit=400), "C1 FP64")


def test_fp64_c2_several_ranges(ctx):
    """More than 64 steps: the solve crosses graph ranges (one graph each)."""
    c = synth.make_config("C2")
    p, me, mi = _problem(ctx, c, B.C128)
    a, b = _both(p, c["dirs"], tol=1e-9, maxit=2000)
    assert a[1]["iterations"] > 2 * 64
    _same(a, b, "C2 FP64")


def test_mixed_single(ctx):
    c = synth.make_config("C1")
    p, me, mi = _problem(ctx, c, B.C64_MIXED)
    _same(*_both(p, c["dirs"], tol=1e-10, maxit=400), "C1 mixed")


def test_block_runs(ctx):
    """Eight directions in one matrix-core block (runs finishing at
    different steps)."""
    (xe, te), (xi, ti), rng = synth.make_pair(3, 3, "fib", 0.01, (1.0, 0.8, 0.6), int_n=700)
    c = dict(ext=(xe, te), int=(xi, ti), k_ext=6.0, k_int=12.0, rho_ext=1.0, rho_int=2.0)
    p, me, mi = _problem(ctx, c, B.C64_MIXED)
    dirs = synth.plane_wave_directions(8, rng)
    _same(*_both(p, dirs, tol=1e-8, maxit=1000, batch=8), "block of 8")


def test_pmchwt(ctx):
    c = synth.make_config("C1")
    p, me, mi = _problem(ctx, c, B.C128)
    p.set_graphs(False)
    xe, se, ce = p.solve_pmchwt(c["dirs"], tol=1e-11, maxit=400)
    p.set_graphs(True)
    xg, sg, cg = p.solve_pmchwt(c["dirs"], tol=1e-11, maxit=400)
    _same((xe.cpu().numpy(), {**se, "ir_steps": 0}, ce), (xg.cpu().numpy(), {**sg, "ir_steps": 0}, cg), "PMCHWT")


def test_side_stream_and_replays():
    """A context on a torch side stream; three graph solves in a row with
    eager device work and host synchronisations between them, each equal to
    the solve launched one by one."""
    s = torch.cuda.Stream()
    ctx = B.Context(0, stream=s)
    c = synth.make_config("C1")
    with torch.cuda.stream(s):
        p, me, mi = _problem(ctx, c, B.C128)
        p.set_graphs(False)
        ref, sref, _ = p.solve(c["dirs"], tol=1e-12, maxit=400)
        ref = ref.cpu().numpy()
        p.set_graphs(True)
        for rep in range(3):
            junk = torch.randn(1 << 20, device="cuda").sum()   # other device work between the replays
            torch.cuda.synchronize()
            x, st, code = p.solve(c["dirs"], tol=1e-12, maxit=400)
            assert code == B.OK and st["graph_steps"] > 0
            assert np.array_equal(x.cpu().numpy(), ref), rep
            assert float(junk) == float(junk)
    del p, me, mi
    ctx.close()


def test_bad_argument(ctx):
    c = synth.make_config("C1")
    p, me, mi = _problem(ctx, c, B.C128)
    from paper_2206_00708_amd import _native as N, api as A
    with pytest.raises(B.BemError):
        A._check(N.load().bem_problem_set_graphs(p._h, 2))
