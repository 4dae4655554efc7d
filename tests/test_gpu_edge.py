"""GPU edge cases through the C ABI: degenerate and limiting configurations
of the method, checked against the oracle (tolerances as in the parity
tests: operators 1e-12 (FP64), mortar 1e-14, traces 1e-5)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

B = pytest.importorskip("paper_2206_00708_amd")


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def ctx():
    assert torch.cuda.is_available(), "GPU tests need a device"
    return B.Context(0)


def _problem(ctx, ext, inte, ke, ki, re=1.0, ri=1.0, prec=B.C128):
    me, mi = B.Mesh(ctx, *ext), B.Mesh(ctx, *inte)
    p = B.Problem(ctx, me, mi, ke, ki, re, ri, precision=prec)
    p.assemble_operators()
    p.assemble_projection()
    return p, me, mi


def _blocks(x, ne, ni):
    return (x[:ne], x[ne:2 * ne], x[2 * ne:2 * ne + ni], x[2 * ne + ni:])


@pytest.mark.parametrize("prec", [B.C128, B.C64_MIXED])
def test_transparent_body(ctx, orc, prec):
    """k_int = k_ext and equal densities: the body is invisible.  The solve
    matches the oracle's LU solution, and -v_ext is the incident wave at the
    exterior nodes up to the discretisation error."""
    c = synth.make_config("C1")
    p, _, _ = _problem(ctx, c["ext"], c["int"], 2.0, 2.0, prec=prec)
    d = np.array([[0.0, 0.6, 0.8]])
    X, _ = orc.solve_mtf(c["ext"], c["int"], 2.0, 2.0, 1.0, 1.0, d)
    out, st, code = p.solve(d, tol=1e-9, maxit=600)
    assert code == B.OK, st
    x = out.cpu().numpy()[0]
    ne, ni = len(c["ext"][0]), len(c["int"][0])
    for g, r in zip(_blocks(x, ne, ni), _blocks(X[0], ne, ni)):
        assert _rel(g, r) < 1e-5
    u = np.exp(1j * 2.0 * c["ext"][0] @ d[0])
    assert _rel(-x[:ne], u) < 0.05


def test_identical_meshes_projection_is_mass(ctx, orc):
    """One mesh for both sides (the conforming limit): the mortar matrix is
    the mass matrix, to rounding."""
    xyz, tri = synth.icosphere(2)
    p, _, _ = _problem(ctx, (xyz, tri), (xyz, tri), 2.0, 3.0)
    import scipy.sparse as sp
    rp, col, val = p.projection()
    P = sp.csr_matrix((val, col, rp), shape=(len(xyz), len(xyz))).toarray()
    M = orc.mass(xyz, tri)
    assert np.abs(P - M).max() < 1e-14 * np.abs(M).max()


def test_maxit_one(ctx):
    c = synth.make_config("C1")
    for prec, batch in ((B.C128, 0), (B.C64_MIXED, 0), (B.C64_MIXED, 3)):
        p, _, _ = _problem(ctx, c["ext"], c["int"], c["k_ext"], c["k_int"], prec=prec)
        d = synth.plane_wave_directions(3, np.random.default_rng(8))
        out, st, code = p.solve(d, tol=1e-12, maxit=1, ir_max=1, batch=batch)
        assert code == B.W_NOCONV
        assert 1 <= st["iterations"] <= 3
        assert np.all(np.isfinite(out.cpu().numpy()))


def test_batches_beyond_64(ctx):
    """70 directions with batch 64: two groups (64 + 6 runs); columns of both
    groups equal their one-at-a-time solves."""
    c = synth.make_config("C1")
    p, _, _ = _problem(ctx, c["ext"], c["int"], c["k_ext"], c["k_int"], prec=B.C64_MIXED)
    d = synth.plane_wave_directions(70, np.random.default_rng(9))
    out, st, code = p.solve(d, tol=1e-8, maxit=400, batch=64)
    assert code == B.OK, st
    pick = [0, 63, 64, 69]
    seq, s1, c1 = p.solve(d[pick], tol=1e-8, maxit=400)
    assert c1 == B.OK
    got, sq = out.cpu().numpy(), seq.cpu().numpy()
    for q, r in enumerate(pick):
        assert _rel(got[r], sq[q]) < 1e-6, r


def test_tetrahedron_matrix_cores(ctx, orc):
    """Four vertices per mesh (GEMM tiles far larger than the matrices, one K
    stage): batched products and a batched solve against the oracle."""
    xyz = np.array([[1.0, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]]) * 0.5
    tri = synth.orient_outward(xyz, np.array([[0, 1, 2], [0, 1, 3], [0, 2, 3], [1, 2, 3]], dtype=np.int32))
    p, _, _ = _problem(ctx, (xyz, tri), (xyz, tri), 1.3, 2.1, prec=B.C64_MIXED)
    ops = orc.operators((xyz, tri), (xyz, tri), 1.3, 2.1)
    A = orc.mtf_system(ops, 1.0, 1.0)
    rng = np.random.default_rng(10)
    X = rng.standard_normal((3, 16)) + 1j * rng.standard_normal((3, 16))
    Y = p.mtf_matvec_batch(torch.from_numpy(X), strong=False).cpu().numpy()
    for r in range(3):
        assert _rel(Y[r], A @ X[r]) < 2e-5
    d = synth.plane_wave_directions(3, rng)
    Xs, _ = orc.solve_mtf((xyz, tri), (xyz, tri), 1.3, 2.1, 1.0, 1.0, d, ops=ops)
    out, st, code = p.solve(d, tol=1e-9, maxit=64, batch=3)
    assert code == B.OK, st
    got = out.cpu().numpy()
    for r in range(3):
        assert _rel(got[r], Xs[r]) < 1e-5


def test_released_blocks_reused_and_trimmed():
    """Released device blocks are kept by the context and handed out again:
    a second identical solve gives the same traces bit for bit and holds no
    more device memory than the first; bem_ctx_trim returns every byte of a
    context whose meshes and problems are gone.  Under a budget that the
    cache would exceed, cached blocks are dropped instead of failing."""
    small = synth.make_config("C1")
    ext, inte, _ = synth.make_pair(11, 3, "fib", 0.01, (1.0, 1.0, 1.0), int_n=500)
    big = {"ext": ext, "int": inte, "k_ext": 3.0, "k_int": 5.0, "rho_ext": 1.0, "rho_int": 1.5}
    d = np.array([[0.0, 0.0, 1.0]])

    def run(cx, c):
        p, me, mi = _problem(cx, c["ext"], c["int"], c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"])
        out, st, code = p.solve(d, tol=1e-8, maxit=300)
        assert code == B.OK, st
        x, used = out.cpu().numpy(), cx.bytes_in_use()
        p.close(); me.close(); mi.close()
        return x, used

    cx = B.Context(0)
    x1, used1 = run(cx, small)
    x2, used2 = run(cx, small)
    assert np.array_equal(x1, x2)
    assert used2 <= used1
    assert cx.bytes_in_use() > 0   # released blocks and the assembly scratch are still held
    cx.trim()
    assert cx.bytes_in_use() == 0
    xb, used_big = run(cx, big)
    cx.trim()
    cx.close()
    # small then big under a budget that both fit only if the small problem's cached blocks are dropped
    assert used_big > used1
    budget = used_big + used1 // 2
    cb = B.Context(0, hbm_budget_bytes=budget)
    xs, _ = run(cb, small)
    xb2, _ = run(cb, big)
    assert np.array_equal(xs, x1) and np.array_equal(xb2, xb)
    assert cb.bytes_in_use() <= budget
    cb.close()


def test_projection_before_operators_same_traces():
    """bem_assemble_projection runs on the context's second stream; called
    before bem_assemble_operators (or after it, the usual order) it must give
    the same solve, bit for bit."""
    c = synth.make_config("C1")
    d = np.array([[0.0, 0.0, 1.0]])
    cx = B.Context(0)
    outs = []
    for first_projection in (False, True):
        me, mi = B.Mesh(cx, *c["ext"]), B.Mesh(cx, *c["int"])
        p = B.Problem(cx, me, mi, c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"])
        if first_projection:
            p.assemble_projection()
            p.assemble_operators()
        else:
            p.assemble_operators()
            p.assemble_projection()
        out, st, code = p.solve(d, tol=1e-8, maxit=300)
        assert code == B.OK, st
        outs.append(out.cpu().numpy())
        p.close(); me.close(); mi.close()
    assert np.array_equal(outs[0], outs[1])
    cx.close()
