"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs.  FP64 path tolerances: operators 1e-12 relative (Frobenius
and entrywise against the largest entry), mortar 1e-14, mat-vecs 1e-12,
traces 1e-5 relative (the target of the method), all stated per test."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2206_00708_amd")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _relmax(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a device"
    return B.Context(0)


def _problem(ctx, c, ng=4):
    me = B.Mesh(ctx, *c["ext"])
    mi = B.Mesh(ctx, *c["int"])
    p = B.Problem(ctx, me, mi, c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"], singular_gauss=ng)
    return p, me, mi


@pytest.fixture(scope="module")
def c1(ctx):
    c = synth.make_config("C1")
    p, me, mi = _problem(ctx, c)
    p.assemble_operators()
    p.assemble_projection()
    return c, p, me, mi


@pytest.fixture(scope="module")
def c1_oracle(orc):
    c = synth.make_config("C1")
    return orc.operators(c["ext"], c["int"], c["k_ext"], c["k_int"])


@pytest.mark.parametrize("mesh", [0, 1])
def test_operators_c1(c1, c1_oracle, mesh):
    c, p, _, _ = c1
    ref = c1_oracle["ext" if mesh == 0 else "int"]
    for op in "VKTD":
        got = p.operator(mesh, op).cpu().numpy()
        assert _rel(got, ref[op]) < 1e-12, (op, _rel(got, ref[op]))
        assert _relmax(got, ref[op]) < 1e-12, op


@pytest.mark.parametrize("k", [0.5, 4.0, 12.0])
def test_operators_phase_paths(ctx, orc, k):
    """The regular kernel evaluates exp(i k r) from a per-pair base phase when
    k times the two triangles' quadrature radii is at most 1, and by the
    reduced sin/cos otherwise: on the C1 exterior mesh (radius about 0.13)
    k = 0.5 takes the first path for every pair, k = 12 the second, k = 4
    mixes them.  Against the oracle at the FP64 operator tolerance."""
    c = synth.make_config("C1")
    me, mi = B.Mesh(ctx, *c["ext"]), B.Mesh(ctx, *c["int"])
    p = B.Problem(ctx, me, mi, k, k, 1.0, 1.0)
    p.assemble_operators()
    ref = orc.assemble(*c["ext"], k)
    for op in "VKTD":
        got = p.operator(0, op).cpu().numpy()
        assert _rel(got, ref[op]) < 1e-12, (k, op, _rel(got, ref[op]))
        assert _relmax(got, ref[op]) < 1e-12, (k, op)


@pytest.mark.parametrize("parts", [1, 2])
def test_operator_parts_c1(ctx, orc, parts):
    """Regular-only and singular-only contributions separately."""
    c = synth.make_config("C1")
    p, me, mi = _problem(ctx, c)
    p.assemble_operators(parts)
    ref = orc.assemble(*c["ext"], c["k_ext"], which=parts)
    for op in "VKTD":
        got = p.operator(0, op).cpu().numpy()
        assert _rel(got, ref[op]) < 1e-12, (parts, op)


def test_projection_c1(c1, c1_oracle):
    import scipy.sparse as sp
    c, p, _, _ = c1
    rp, col, val = p.projection()
    P = sp.csr_matrix((val, col, rp), shape=(len(c["int"][0]), len(c["ext"][0]))).toarray()
    ref = c1_oracle["P_ie"]
    assert np.abs(P - ref).max() < 1e-14 * np.abs(ref).max()


def test_rhs_c1(c1, orc):
    c, p, _, _ = c1
    b = p.mtf_rhs(c["dirs"]).cpu().numpy()[0]
    ref = orc.mtf_rhs(c["ext"], c["k_ext"], c["dirs"][0], len(c["int"][0]))
    assert _relmax(b, ref) < 1e-13


@pytest.mark.parametrize("strong", [False, True])
def test_matvec_c1(c1, c1_oracle, orc, strong):
    c, p, _, _ = c1
    A = orc.mtf_system(c1_oracle, c["rho_ext"], c["rho_int"])
    rng = np.random.default_rng(5)
    x = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    y = p.mtf_matvec(torch.from_numpy(x), strong=strong).cpu().numpy()
    ref = A @ x
    if strong:
        ref = np.linalg.solve(orc.block_mass(c1_oracle), ref)
    assert _rel(y, ref) < 1e-12


def test_solve_c1_vs_lu(c1, c1_oracle, orc):
    c, p, _, _ = c1
    X, _ = orc.solve_mtf(c["ext"], c["int"], c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"], c["dirs"],
                         ops=c1_oracle)
    out, stats, code = p.solve(c["dirs"], tol=c["tol"], maxit=500)
    assert code == B.OK
    got = out.cpu().numpy()[0]
    ne, ni = len(c["ext"][0]), len(c["int"][0])
    for sl in (slice(0, ne), slice(ne, 2 * ne), slice(2 * ne, 2 * ne + ni), slice(2 * ne + ni, None)):
        assert _rel(got[sl], X[0][sl]) < 1e-5
    assert stats["rel_residual"] < 10 * c["tol"]
    assert stats["iterations"] > 0


def test_bitwise_repeatable(ctx):
    c = synth.make_config("C1")
    p, me, mi = _problem(ctx, c)
    p.assemble_operators()
    a = [p.operator(0, op).clone() for op in "VKTD"]
    p.assemble_operators()
    b = [p.operator(0, op) for op in "VKTD"]
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_tetrahedron_all_pairs_singular(ctx, orc):
    """Smallest closed mesh: every triangle pair shares an edge."""
    xyz = np.array([[1.0, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]]) * 0.5
    tri = synth.orient_outward(xyz, np.array([[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]], dtype=np.int32))
    me = B.Mesh(ctx, xyz, tri)
    p = B.Problem(ctx, me, me, 1.3, 2.1, 1.0, 1.0)
    p.assemble_operators()
    ref = orc.assemble(xyz, tri, 1.3)
    for op in "VKTD":
        assert _rel(p.operator(0, op).cpu().numpy(), ref[op]) < 1e-12


@pytest.mark.parametrize("ng", [1, 3, 6])
def test_singular_orders(ctx, orc, ng):
    xyz, tri = synth.icosphere(1)
    me = B.Mesh(ctx, xyz, tri)
    p = B.Problem(ctx, me, me, 2.0, 3.0, 1.0, 1.0, singular_gauss=ng)
    p.assemble_operators()
    ref = orc.assemble(xyz, tri, 3.0, ng=ng)
    for op in "VKTD":
        assert _rel(p.operator(1, op).cpu().numpy(), ref[op]) < 1e-12


def test_error_paths(ctx):
    c = synth.make_config("C1")
    me = B.Mesh(ctx, *c["ext"])
    mi = B.Mesh(ctx, *c["int"])
    with pytest.raises(B.BemError) as e:
        B.Problem(ctx, me, mi, -1.0, 2.0)
    assert e.value.code == -1
    p = B.Problem(ctx, me, mi, 2.0, 4.0)
    with pytest.raises(B.BemError) as e:
        p.solve([[0, 0, 1.0]])
    assert e.value.code == -4
    p.assemble_operators()
    p.assemble_projection()
    out, stats, code = p.solve([[0, 0, 1.0]], tol=1e-14, maxit=3)
    assert code == B.W_NOCONV and stats["iterations"] == 3
    with pytest.raises(B.BemError):
        B.Mesh(ctx, c["ext"][0], c["ext"][1][1:])


# ---------------------------------------------------------------- full size

@pytest.fixture(scope="module")
def c2(ctx):
    c = synth.make_config("C2")
    p, me, mi = _problem(ctx, c)
    p.assemble_operators()
    p.assemble_projection()
    return c, p, me, mi


def _sample_rows(nv, rng, k=6):
    return np.unique(np.concatenate([[0, nv - 1], rng.choice(nv, k, replace=False)]))


@pytest.mark.parametrize("mesh", [0, 1])
def test_operators_c2_sampled_rows(c2, orc, mesh):
    c, p, _, _ = c2
    xyz, tri = c["ext"] if mesh == 0 else c["int"]
    k = c["k_ext"] if mesh == 0 else c["k_int"]
    rows = _sample_rows(len(xyz), np.random.default_rng(mesh))
    ref = orc.assemble(xyz, tri, k, rows=rows)
    for op in "VKTD":
        got = p.operator(mesh, op)[torch.from_numpy(rows).cuda()].cpu().numpy()
        assert _rel(got, ref[op]) < 1e-12, op


def test_projection_c2_sampled_rows(c2, orc):
    import scipy.sparse as sp
    c, p, _, _ = c2
    rp, col, val = p.projection()
    P = sp.csr_matrix((val, col, rp), shape=(len(c["int"][0]), len(c["ext"][0])))
    rows = _sample_rows(len(c["int"][0]), np.random.default_rng(7), 20)
    ref = orc.mortar(c["int"], c["ext"], rows=rows)
    assert np.abs(P[rows].toarray() - ref).max() < 1e-14 * np.abs(ref).max()
    # partition of unity: column sums equal the exterior lumped mass
    Me = orc.mass(*c["ext"])
    assert np.abs(np.asarray(P.sum(0)).ravel() - Me.sum(1)).max() < 1e-14


# Full-size trace parity (C2 solve against the oracle's exact discrete
# solution) is in test_gpu_golden.py.


@pytest.mark.parametrize("strip_tiles", [1, 37, 400])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_operators_strips(orc, strip_tiles, prec):
    """The regular-pair assembly strip by strip: a context whose meshes take
    tiny strips (one block row each, 37 tiles, 400 tiles) on the small
    ellipsoid pair (642 / 700 vertices: about 80 blocks per mesh, so up to
    80 strips, with entries fed by several strips summed strip by strip),
    every entry of V, K, T, D of both meshes against the oracle: 1e-12 in
    FP64, 2e-5 for the complex64 operators (the mixed form's tolerance)."""
    ctx = B.Context(0)
    ctx.set_strip_tiles(strip_tiles)
    (xe, te), (xi, ti), _ = synth.make_pair(3, 3, "fib", 0.01, (1.0, 0.8, 0.6), int_n=700)
    me, mi = B.Mesh(ctx, xe, te), B.Mesh(ctx, xi, ti)
    p = B.Problem(ctx, me, mi, 6.0, 12.0, 1.0, 2.0, precision=B.C128 if prec == "fp64" else B.C64_MIXED)
    p.assemble_operators()
    bound = 1e-12 if prec == "fp64" else 2e-5
    for mesh, (x, t, k) in enumerate(((xe, te, 6.0), (xi, ti, 12.0))):
        ref = orc.assemble(x, t, k)
        for op in "VKTD":
            got = p.operator(mesh, op).cpu().numpy().astype(np.complex128)
            e, em = _rel(got, ref[op]), _relmax(got, ref[op])
            assert e < bound and em < bound, (strip_tiles, mesh, op, e, em)
    del p, me, mi
    ctx.close()


@pytest.mark.parametrize("strip_tiles", [0, 37])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_regular_part_exactly_symmetric(strip_tiles, prec):
    """The regular-pair part alone (no vertex-sharing pairs) on the small
    ellipsoid pair, in one strip per mesh and in strips of 37 tiles: every
    unordered vertex pair is summed once and written in both orientations,
    so V and D equal their transposes and K equals T transposed, bitwise
    (Sec. 2.1: V and D are symmetric and K' is the adjoint of K under the
    Galerkin pairing)."""
    ctx = B.Context(0)
    ctx.set_strip_tiles(strip_tiles)
    (xe, te), (xi, ti), _ = synth.make_pair(3, 3, "fib", 0.01, (1.0, 0.8, 0.6), int_n=700)
    me, mi = B.Mesh(ctx, xe, te), B.Mesh(ctx, xi, ti)
    p = B.Problem(ctx, me, mi, 6.0, 12.0, 1.0, 2.0, precision=B.C128 if prec == "fp64" else B.C64_MIXED)
    p.assemble_operators(parts=1)
    for mesh in (0, 1):
        V, K, T, D = (p.operator(mesh, op).cpu().numpy() for op in "VKTD")
        assert np.abs(V).max() > 0 and np.abs(K).max() > 0
        assert np.array_equal(V, V.T), mesh
        assert np.array_equal(D, D.T), mesh
        assert np.array_equal(K, T.T), mesh
    del p, me, mi
    ctx.close()
