"""Point-source incident field (Sec. 5.7) through the C ABI against the
oracle: loads to 1e-13 (as the plane-wave loads), the solve against the
oracle's LU solution to 1e-5, the field to 1e-11, and argument checks."""
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


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _c1(ctx):
    c = synth.make_config("C1")
    me, mi = B.Mesh(ctx, *c["ext"]), B.Mesh(ctx, *c["int"])
    p = B.Problem(ctx, me, mi, c["k_ext"], c["k_int"], 1.0, 1.5)
    p.assemble_operators()
    p.assemble_projection()
    p.set_incident(1)
    return c, p, me, mi


def test_point_source_loads_match_oracle(ctx, orc):
    c, p, me, mi = _c1(ctx)
    srcs = np.array([[0.3, -0.2, 2.5], [-1.7, 0.4, -0.9]])
    b = p.mtf_rhs(srcs).cpu().numpy()
    ne, ni = len(c["ext"][0]), len(c["int"][0])
    for r in range(2):
        ref = orc.mtf_rhs(c["ext"], c["k_ext"], srcs[r], ni, incident=1)
        assert np.abs(b[r] - ref).max() < 1e-13 * np.abs(ref).max()


def test_point_source_solve_and_field_match_oracle(ctx, orc):
    from oracle import field as F
    c, p, me, mi = _c1(ctx)
    srcs = np.array([[0.3, -0.2, 2.5]])
    out, st, code = p.solve(srcs, tol=1e-10, maxit=600)
    assert code == B.OK, st
    X, _ = orc.solve_mtf(c["ext"], c["int"], c["k_ext"], c["k_int"], 1.0, 1.5, srcs, incident=1)
    assert _rel(out.cpu().numpy()[0], X[0]) < 1e-5
    g = np.linspace(-1.8, 1.8, 13)
    gx, gy = np.meshgrid(g, g, indexing="ij")
    pts = np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, 0.1)], axis=1)
    region = (F.winding(*c["ext"], pts) > 0.5).astype(np.int32)
    x = torch.as_tensor(X)
    got = p.field(srcs, x, pts, torch.as_tensor(region)).cpu().numpy()[0]
    ref = F.mtf_field(c["ext"], c["int"], c["k_ext"], c["k_int"], X[0], srcs[0], pts, region, kind=1)
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-11


def test_incident_kind_checks(ctx):
    c, p, me, mi = _c1(ctx)
    with pytest.raises(B.BemError):
        p.set_incident(2)
    with pytest.raises(B.BemError):
        p.solve(np.array([[np.nan, 0.0, 0.0]]))
    p.set_incident(0)
    with pytest.raises(B.BemError):
        p.solve(np.array([[0.3, -0.2, 2.5]]))   # not a unit direction
