"""Mortar matrix with its geometry on the device (Sec. 3.1) through the C ABI:
against the oracle's dense mortar (C1, an ellipsoid pair, identical meshes)
to 1e-14 of the largest entry, against the host assembly at C3 (same
sparsity, values to 1e-14), the solve with either setting, the coverage check
on meshes that do not match, and the argument checks."""
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


def _dense(p, ni, ne):
    import scipy.sparse as sp
    rp, col, val = p.projection()
    return sp.csr_matrix((val, col, rp), shape=(ni, ne)).toarray(), (rp, col, val)


def _problem(ctx, ext, inte, on_device, k=(5.0, 8.0)):
    me, mi = B.Mesh(ctx, *ext), B.Mesh(ctx, *inte)
    p = B.Problem(ctx, me, mi, k[0], k[1], 1.0, 1.5)
    p.set_mortar(on_device)
    p.assemble_projection()
    return p, me, mi


def _ellipsoid():
    ext, inte, _ = synth.configs.make_pair(11, 3, "fib", 0.02, (1.0, 0.8, 0.6), int_n=700)
    return ext, inte


@pytest.mark.parametrize("case", ["C1", "ellipsoid", "identical"])
def test_device_mortar_matches_oracle(ctx, orc, case):
    if case == "C1":
        c = synth.make_config("C1")
        ext, inte = c["ext"], c["int"]
    elif case == "ellipsoid":
        ext, inte = _ellipsoid()
    else:
        c = synth.make_config("C1")
        ext = inte = c["ext"]
    p, _, _ = _problem(ctx, ext, inte, True)
    P, _ = _dense(p, len(inte[0]), len(ext[0]))
    ref = orc.mortar(inte, ext)
    assert np.abs(P - ref).max() < 1e-14 * np.abs(ref).max(), case
    assert p.mortar_ms() > 0.0


def test_device_mortar_equals_host_c3(ctx):
    c = synth.make_config("C3")
    ph, _, _ = _problem(ctx, c["ext"], c["int"], False, (c["k_ext"], c["k_int"]))
    pd, _, _ = _problem(ctx, c["ext"], c["int"], True, (c["k_ext"], c["k_int"]))
    rh, ch, vh = ph.projection()
    rd, cd, vd = pd.projection()
    assert np.array_equal(rh, rd) and np.array_equal(ch, cd)
    assert np.abs(vh - vd).max() < 1e-14 * np.abs(vh).max()
    print(f"C3 mortar: host {ph.mortar_ms():.2f} ms, device {pd.mortar_ms():.2f} ms")


def test_solve_with_device_mortar(ctx):
    c = synth.make_config("C1")
    out = []
    for on in (False, True):
        me, mi = B.Mesh(ctx, *c["ext"]), B.Mesh(ctx, *c["int"])
        p = B.Problem(ctx, me, mi, c["k_ext"], c["k_int"], 1.0, 1.5)
        p.set_mortar(on)
        p.assemble_operators()
        p.assemble_projection()
        x, st, code = p.solve(c["dirs"], tol=1e-10, maxit=600)
        assert code == B.OK, st
        out.append(x.cpu().numpy())
    assert np.linalg.norm(out[0] - out[1]) < 1e-10 * np.linalg.norm(out[0])


def test_device_mortar_checks(ctx):
    c = synth.make_config("C1")
    xi, ti = c["int"]
    me, mi = B.Mesh(ctx, *c["ext"]), B.Mesh(ctx, xi * 0.5 + np.array([2.0, 0.0, 0.0]), ti)
    p = B.Problem(ctx, me, mi, 5.0, 8.0, 1.0, 1.5)
    with pytest.raises(B.BemError):
        p.set_mortar(2)
    with pytest.raises(B.BemError):
        p.mortar_ms()
    p.set_mortar(True)
    with pytest.raises(B.BemError):     # the shifted interior mesh leaves the exterior facets uncovered
        p.assemble_projection()
