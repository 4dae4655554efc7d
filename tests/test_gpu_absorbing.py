"""Absorbing interior (the foam model of Sec. 5.7: a complex interior
wavenumber k_int + i k_im) through the C ABI against the oracle, which
evaluates exp(i k r) / (4 pi r) with the complex k itself: interior operators
to 1e-12 (FP64) and to the complex64 bounds of the mixed path, the exterior
operators untouched, the multiple-traces and PMCHWT solves against the
oracle's LU solutions, the interior field, and the argument and state
checks."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2206_00708_amd")

K_IM = 0.6
OP_FRO, OP_MAX = 2e-5, 1e-4     # complex64 storage, as the lossless mixed-precision operators


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a device"
    return B.Context(0)


@pytest.fixture(scope="module")
def c1():
    return synth.make_config("C1")


@pytest.fixture(scope="module")
def c1_ops(orc, c1):
    return orc.operators(c1["ext"], c1["int"], c1["k_ext"], c1["k_int"] + 1j * K_IM)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _relmax(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def _problem(ctx, c, precision=B.C128):
    me, mi = B.Mesh(ctx, *c["ext"]), B.Mesh(ctx, *c["int"])
    p = B.Problem(ctx, me, mi, c["k_ext"], c["k_int"], 1.0, 1.5, precision=precision)
    p.set_k_int_imag(K_IM)
    p.assemble_operators()
    p.assemble_projection()
    return p, me, mi


def test_absorbing_operators_fp64(ctx, c1, c1_ops):
    p, _, _ = _problem(ctx, c1)
    for mesh, key in ((0, "ext"), (1, "int")):
        for op in "VKTD":
            got = p.operator(mesh, op).cpu().numpy()
            ref = c1_ops[key][op]
            assert _rel(got, ref) < 1e-12 and _relmax(got, ref) < 1e-12, (key, op, _rel(got, ref))


def test_absorbing_operators_mixed(ctx, c1, c1_ops):
    p, _, _ = _problem(ctx, c1, B.C64_MIXED)
    for op in "VKTD":
        got = p.operator(1, op).cpu().numpy().astype(np.complex128)
        ref = c1_ops["int"][op]
        e, m = _rel(got, ref), _relmax(got, ref)
        print(f"absorbing mixed {op}: fro {e:.2e} max {m:.2e}")
        assert e < OP_FRO and m < OP_MAX, (op, e, m)


def test_absorbing_solve_and_field(ctx, orc, c1, c1_ops):
    from oracle import field as F
    p, _, _ = _problem(ctx, c1)
    d = np.array([[0.0, 0.6, 0.8]])
    out, st, code = p.solve(d, tol=1e-10, maxit=600)
    assert code == B.OK, st
    ki = c1["k_int"] + 1j * K_IM
    X, _ = orc.solve_mtf(c1["ext"], c1["int"], c1["k_ext"], ki, 1.0, 1.5, d, ops=c1_ops)
    assert _rel(out.cpu().numpy()[0], X[0]) < 1e-5
    g = np.linspace(-1.8, 1.8, 13)
    gx, gy = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, 0.1)], axis=1)
    region = (F.winding(*c1["ext"], pts) > 0.5).astype(np.int32)
    assert 0 < region.sum() < region.size
    got = p.field(d, torch.as_tensor(X), pts, torch.as_tensor(region)).cpu().numpy()[0]
    ref = F.mtf_field(c1["ext"], c1["int"], c1["k_ext"], ki, X[0], d[0], pts, region)
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-11


def test_absorbing_pmchwt(ctx, orc, c1, c1_ops):
    p, _, _ = _problem(ctx, c1)
    d = np.array([[0.0, 0.0, 1.0]])
    out, st, code = p.solve_pmchwt(d, tol=1e-10, maxit=400)
    assert code == B.OK, st
    X, _ = orc.solve_pmchwt(c1["ext"], c1["int"], c1["k_ext"], c1["k_int"] + 1j * K_IM, 1.0, 1.5, d,
                            ops=c1_ops)
    assert _rel(out.cpu().numpy()[0], X[0]) < 1e-5


def test_absorption_checks_and_stale_operators(ctx, c1):
    p, _, _ = _problem(ctx, c1)
    for bad in (-0.1, float("nan"), float("inf")):
        with pytest.raises(B.BemError):
            p.set_k_int_imag(bad)
    p.set_k_int_imag(K_IM)                      # unchanged: the operators stay valid
    p.solve(np.array([[0.0, 0.0, 1.0]]), tol=1e-6, maxit=200)
    p.set_k_int_imag(0.0)                       # changed: assemble again first
    with pytest.raises(B.BemError):
        p.solve(np.array([[0.0, 0.0, 1.0]]), tol=1e-6, maxit=200)
    p.assemble_operators()
    out, st, code = p.solve(np.array([[0.0, 0.0, 1.0]]), tol=1e-6, maxit=200)
    assert code == B.OK


def test_absorbing_solve_mixed(ctx, orc, c1, c1_ops):
    """The mixed form end to end (complex64 operators from the FP32
    complex-wavenumber kernel, FP64 refinement) against the oracle's LU
    solution, to the same 1e-5 as the lossless mixed solves."""
    p, _, _ = _problem(ctx, c1, B.C64_MIXED)
    d = np.array([[0.0, 0.6, 0.8]])
    out, st, code = p.solve(d, tol=c1["tol"], maxit=500)
    assert code == B.OK, st
    X, _ = orc.solve_mtf(c1["ext"], c1["int"], c1["k_ext"], c1["k_int"] + 1j * K_IM, 1.0, 1.5, d, ops=c1_ops)
    assert _rel(out.cpu().numpy()[0], X[0]) < 1e-5
