"""Field evaluation and winding numbers through the C ABI against the
oracle's representation-formula sums (FP64: the same 6-point sums in a
different order, so the bar is rounding: 1e-11 of the largest value) and
against the oracle's winding numbers (1e-12)."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2206_00708_amd")
N = pytest.importorskip("paper_2206_00708_amd._native")


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a device"
    return B.Context(0)


@pytest.fixture(scope="module")
def F():
    from oracle import field
    return field


def _problem(ctx, name):
    c = synth.make_config(name)
    me, mi = B.Mesh(ctx, *c["ext"]), B.Mesh(ctx, *c["int"])
    p = B.Problem(ctx, me, mi, c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"])
    p.assemble_operators()
    p.assemble_projection()
    return c, p, me, mi


def _grid(nx, ny, half, z):
    """nx x ny points in the square [-half, half]^2 of the plane z."""
    gx, gy = np.meshgrid(np.linspace(-half, half, nx), np.linspace(-half, half, ny), indexing="ij")
    return np.stack([gx.ravel(), gy.ravel(), np.full(gx.size, z)], axis=1)


def _random_unknowns(n, nrhs, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nrhs, n)) + 1j * rng.standard_normal((nrhs, n))


def _check_field(F, c, p, x, dirs, pts, region, tol=1e-11):
    got = p.field(dirs, torch.as_tensor(x), pts, torch.as_tensor(region)).cpu().numpy()
    for r in range(x.shape[0]):
        ref = F.mtf_field(c["ext"], c["int"], c["k_ext"], c["k_int"], x[r], dirs[r], pts, region)
        err = np.max(np.abs(got[r] - ref)) / np.max(np.abs(ref))
        assert err < tol, (r, err)
    return got


def test_winding_matches_oracle(ctx, F):
    c, p, me, mi = _problem(ctx, "C1")
    rng = np.random.default_rng(1)
    pts = np.concatenate([rng.uniform(-1.6, 1.6, (700, 3)), np.zeros((1, 3))])
    for m, mesh in ((me, c["ext"]), (mi, c["int"])):
        w = m.winding(pts).cpu().numpy()
        ref = F.winding(*mesh, pts)
        assert np.max(np.abs(w - ref)) < 1e-12
    r = np.linalg.norm(pts, axis=1)
    w = me.winding(pts).cpu().numpy()
    assert np.all(np.abs(w[r < 0.8] - 1) < 1e-12) and np.all(np.abs(w[r > 1.2]) < 1e-12)


def test_field_matches_oracle_c1(ctx, F):
    """Ragged point count (667), two right-hand sides, interior and exterior
    points, regions from the exterior winding number."""
    c, p, me, mi = _problem(ctx, "C1")
    pts = _grid(23, 29, 2.0, 0.1)
    region = (F.winding(*c["ext"], pts) > 0.5).astype(np.int32)
    assert 0 < region.sum() < len(region)
    x = _random_unknowns(p.n, 2, 3)
    dirs = synth.plane_wave_directions(2, np.random.default_rng(4))
    _check_field(F, c, p, x, dirs, pts, region)
    # the default region rule is the same winding number
    got = p.field(dirs, torch.as_tensor(x), pts).cpu().numpy()
    ref = p.field(dirs, torch.as_tensor(x), pts, torch.as_tensor(region)).cpu().numpy()
    assert np.array_equal(got, ref)


def test_field_of_a_solve_matches_oracle_solve(ctx, orc, F):
    """End to end at C1: device solve, device field against the oracle's LU
    solution and field (the traces agree to the solve tolerance)."""
    c, p, me, mi = _problem(ctx, "C1")
    d = c["dirs"]
    out, st, code = p.solve(d, tol=1e-10, maxit=600)
    assert code == B.OK, st
    X, _ = orc.solve_mtf(c["ext"], c["int"], c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"], d)
    pts = np.concatenate([_grid(9, 9, 1.8, 0.0), 0.3 * _grid(5, 5, 1.0, 0.2)])
    region = (F.winding(*c["ext"], pts) > 0.5).astype(np.int32)
    got = p.field(d, out, pts, torch.as_tensor(region)).cpu().numpy()[0]
    ref = F.mtf_field(c["ext"], c["int"], c["k_ext"], c["k_int"], X[0], d[0], pts, region)
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-7


def test_field_c2_grid_sampled(ctx, F):
    """The measured configuration: C2 meshes, a 100 x 100 grid on z = 0 over
    [-2, 2]^2, the launch shape of the bench; the oracle on 160 sampled
    points (every interior/exterior mix of the grid rows it hits)."""
    c, p, me, mi = _problem(ctx, "C2")
    pts = _grid(100, 100, 2.0, 0.0)
    region = (me.winding(pts).cpu().numpy() > 0.5).astype(np.int32)
    x = _random_unknowns(p.n, 1, 5)
    dirs = c["dirs"]
    got = p.field(dirs, torch.as_tensor(x), pts, torch.as_tensor(region)).cpu().numpy()[0]
    idx = np.random.default_rng(6).choice(len(pts), 160, replace=False)
    ref = F.mtf_field(c["ext"], c["int"], c["k_ext"], c["k_int"], x[0], dirs[0], pts[idx], region[idx])
    assert np.max(np.abs(got[idx] - ref)) / np.max(np.abs(ref)) < 1e-11
    wref = F.winding(*c["ext"], pts[idx])
    assert np.array_equal(region[idx], (wref > 0.5).astype(np.int32))


def test_field_host_memspace_and_edges(ctx):
    """Host buffers give the device result bit for bit; zero points do
    nothing; bad regions and directions are rejected."""
    c, p, me, mi = _problem(ctx, "C1")
    L = N.load()
    pts = np.ascontiguousarray(_grid(7, 11, 1.5, 0.3))
    region = np.ascontiguousarray((np.linalg.norm(pts, axis=1) < 0.9).astype(np.int32))
    x = np.ascontiguousarray(_random_unknowns(p.n, 1, 7))
    d = np.ascontiguousarray(c["dirs"], dtype=np.float64)
    host = np.zeros((1, len(pts)), dtype=np.complex128)
    code = L.bem_field(p._h, d.ctypes.data, 1, x.ctypes.data, pts.ctypes.data, region.ctypes.data, len(pts),
                       host.ctypes.data, B.HOST)
    assert code == B.OK
    dev = p.field(d, torch.as_tensor(x), pts, torch.as_tensor(region)).cpu().numpy()
    assert np.array_equal(host, dev)
    assert L.bem_field(p._h, d.ctypes.data, 1, x.ctypes.data, None, None, 0, None, B.HOST) == B.OK
    bad = region.copy(); bad[3] = 2
    assert L.bem_field(p._h, d.ctypes.data, 1, x.ctypes.data, pts.ctypes.data, bad.ctypes.data, len(pts),
                       host.ctypes.data, B.HOST) == -1   # BEM_E_ARG
    d2 = np.ascontiguousarray(2.0 * d)
    assert L.bem_field(p._h, d2.ctypes.data, 1, x.ctypes.data, pts.ctypes.data, region.ctypes.data, len(pts),
                       host.ctypes.data, B.HOST) == -1   # BEM_E_ARG
    w = np.zeros(len(pts))
    assert L.bem_mesh_winding(me._h, pts.ctypes.data, len(pts), w.ctypes.data, B.HOST) == B.OK
    assert np.array_equal(w, me.winding(pts).cpu().numpy())
