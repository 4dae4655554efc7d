"""The sparse inverse-mass apply (Chebyshev iteration on the Jacobi-scaled
mass matrix over overlapping vertex patches, no dense M^-1) through the C
ABI: the mass-preconditioned product against the oracle's M^-1 A x
(1e-12, the FP64 product tolerance), the solve against the oracle's LU
solution (1e-5 per trace block), agreement with the dense-inverse form, the
automatic choice, and a mesh above the dense form's 16,384-vertex limit,
checked by the defining property M z = y of the strong product (FP64
rounding) with the weak product's sampled rows against the oracle's rows."""
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
    c = B.Context(0)
    yield c
    c.trim()


def _problem(ctx, ext, inte, ke, ki, re, ri, prec=B.C128, mode=2):
    me, mi = B.Mesh(ctx, *ext), B.Mesh(ctx, *inte)
    p = B.Problem(ctx, me, mi, ke, ki, re, ri, precision=prec)
    p.set_mass_apply(mode)
    p.assemble_operators()
    p.assemble_projection()
    return p, me, mi


def _small_ellipsoid():
    (xe, te), (xi, ti), rng = synth.make_pair(3, 3, "fib", 0.01, (1.0, 0.8, 0.6), int_n=700)
    return dict(ext=(xe, te), int=(xi, ti), k_ext=6.0, k_int=12.0, rho_ext=1.0, rho_int=2.0,
                dirs=synth.plane_wave_directions(2, rng))


@pytest.mark.parametrize("case", ["C1", "ellipsoid"])
def test_sparse_strong_product_vs_oracle(ctx, orc, case):
    c = synth.make_config("C1") if case == "C1" else _small_ellipsoid()
    p, me, mi = _problem(ctx, c["ext"], c["int"], c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"])
    assert p.mass_apply_sparse()
    ops = orc.operators(c["ext"], c["int"], c["k_ext"], c["k_int"])
    A = orc.mtf_system(ops, c["rho_ext"], c["rho_int"])
    Mb = orc.block_mass(ops)
    rng = np.random.default_rng(5)
    for _ in range(2):
        x = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
        y = p.mtf_matvec(torch.from_numpy(x), strong=True).cpu().numpy()
        e = _rel(y, np.linalg.solve(Mb, A @ x))
        print(f"{case} sparse strong product: {e:.2e}")
        assert e < 1e-12


def test_sparse_solve_vs_lu(ctx, orc):
    """The smaller twin of the large-mesh test below: the same kind of
    exterior grid (a Fibonacci hull), solved with the sparse apply, against
    the oracle's exact discrete solution."""
    xe, te = synth.meshes.fibonacci_sphere(900)
    te = synth.meshes.orient_outward(xe, te)
    (xi, ti), _, _ = synth.make_pair(8, 3, "ico", 0.01, (1.0, 1.0, 1.0), int_level=3)
    dirs = np.array([[0.0, 0.6, 0.8]])
    p, me, mi = _problem(ctx, (xe, te), (xi, ti), 3.0, 5.0, 1.0, 1.5)
    X, _ = orc.solve_mtf((xe, te), (xi, ti), 3.0, 5.0, 1.0, 1.5, dirs)
    out, st, code = p.solve(dirs, tol=1e-9, maxit=1000)
    assert code == B.OK, st
    got = out.cpu().numpy()[0]
    ne, ni = len(xe), len(xi)
    cuts = [0, ne, 2 * ne, 2 * ne + ni, 2 * ne + 2 * ni]
    errs = [_rel(got[a:b], X[0][a:b]) for a, b in zip(cuts, cuts[1:])]
    print("sparse-apply solve vs LU, per block: " + " ".join(f"{e:.2e}" for e in errs))
    assert max(errs) < 1e-5


def test_preconditioner_steps_same_solution(ctx):
    """Inside GMRES the sparse form preconditions with 12 Chebyshev steps (a
    fixed polynomial p(M) within 7.5e-6 of M^-1, Sec. 3.3 only needs M^-1 as
    the preconditioner of the weak-form system), while the dense form applies
    M^-1 to FP64 rounding.  Both solve A x = b: at a tight tolerance the
    traces of the two agree far below the preconditioner's own error, and
    the step counts match within 2."""
    c = _small_ellipsoid()
    args = (c["ext"], c["int"], c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"])
    pd, a, b = _problem(ctx, *args, mode=1)
    ps, d, e = _problem(ctx, *args, mode=2)
    od, sd, cd = pd.solve(c["dirs"], tol=1e-11, maxit=2000)
    os_, ss, cs = ps.solve(c["dirs"], tol=1e-11, maxit=2000)
    assert cd == B.OK and cs == B.OK
    err = max(_rel(os_.cpu().numpy()[r], od.cpu().numpy()[r]) for r in range(len(c["dirs"])))
    print(f"12-step vs exact M^-1: steps {ss['iterations']} / {sd['iterations']}, trace difference {err:.2e}")
    assert abs(sd["iterations"] - ss["iterations"]) <= 2
    assert err < 1e-9


@pytest.mark.parametrize("prec", [B.C128, B.C64_MIXED], ids=["fp64", "mixed"])
def test_sparse_matches_dense_c2(ctx, prec):
    """Both forms of the apply on the C2 workload: the strong products agree
    to FP64 rounding (FP64 form; the mixed form's dense inverse is stored in
    FP32, so there they agree to its rounding), and the solves take the
    same number of steps with traces within the solve tolerance."""
    c = synth.make_config("C2")
    pd, a, b = _problem(ctx, c["ext"], c["int"], c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"], prec, mode=1)
    ps, d, e = _problem(ctx, c["ext"], c["int"], c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"], prec, mode=2)
    assert ps.mass_apply_sparse() and not pd.mass_apply_sparse()
    rng = np.random.default_rng(9)
    x = torch.from_numpy(rng.standard_normal(pd.n) + 1j * rng.standard_normal(pd.n))
    yd = pd.mtf_matvec(x, strong=True).cpu().numpy()
    ys = ps.mtf_matvec(x, strong=True).cpu().numpy()
    bound = 1e-13 if prec == B.C128 else 1e-6
    print(f"C2 dense vs sparse strong product: {_rel(ys, yd):.2e}")
    assert _rel(ys, yd) < bound
    od, sd, cd = pd.solve(c["dirs"], tol=1e-8, maxit=2000)
    os_, ss, cs = ps.solve(c["dirs"], tol=1e-8, maxit=2000)
    assert cd == B.OK and cs == B.OK
    print(f"C2 steps dense {sd['iterations']} sparse {ss['iterations']}")
    assert abs(sd["iterations"] - ss["iterations"]) <= 2
    assert _rel(os_.cpu().numpy()[0], od.cpu().numpy()[0]) < 1e-6


def test_automatic_choice(ctx):
    c1 = synth.make_config("C1")
    p, me, mi = _problem(ctx, c1["ext"], c1["int"], 2.0, 4.0, 1.0, 1.0, mode=0)
    assert not p.mass_apply_sparse()   # 162 + 162 vertices: the dense inverses are tiny
    p.set_mass_apply(2)
    with pytest.raises(B.BemError):    # the changed mode needs a new projection set-up
        p.solve([[0, 0, 1.0]])
    p.assemble_projection()
    assert p.mass_apply_sparse()
    with pytest.raises(B.BemError):
        p.set_mass_apply(3)


def test_mesh_above_dense_limit(ctx, orc):
    """Exterior Fibonacci hull of 17,000 vertices (more than the dense
    inverse's 16,384), interior icosphere level 3: the automatic choice is
    the sparse apply; the weak product's sampled rows match the oracle's rows
    (1e-12) and the strong product z satisfies M z = y against the oracle's
    mass matrices (FP64 rounding); a solve converges with its true residual
    at the tolerance."""
    xe, te = synth.meshes.fibonacci_sphere(17000)
    te = synth.meshes.orient_outward(xe, te)
    (xi, ti), _, _ = synth.make_pair(8, 3, "ico", 0.01, (1.0, 1.0, 1.0), int_level=3)
    ke, ki, re, ri = 3.0, 5.0, 1.0, 1.5
    p, me, mi = _problem(ctx, (xe, te), (xi, ti), ke, ki, re, ri, mode=0)
    assert p.mass_apply_sparse()
    ne, ni = len(xe), len(xi)
    rng = np.random.default_rng(11)
    x = rng.standard_normal(p.n) + 1j * rng.standard_normal(p.n)
    xt = torch.from_numpy(x)
    y = p.mtf_matvec(xt, strong=False).cpu().numpy()
    z = p.mtf_matvec(xt, strong=True).cpu().numpy()
    rows = np.unique(np.concatenate([[0, ne - 1], rng.choice(ne, 4, replace=False)]))
    Oe = orc.assemble(xe, te, ke, rows=rows)
    Pie = orc.mortar((xi, ti), (xe, te))
    ref = -Oe["K"] @ x[:ne] + Oe["V"] @ x[ne:2 * ne] + 0.5 * Pie.T[rows] @ x[2 * ne:2 * ne + ni]
    e = _rel(y[rows], ref)
    print(f"N_ext {ne}: weak product rows vs oracle {e:.2e}")
    assert e < 1e-12
    Me, Mi = orc.mass(xe, te), orc.mass(xi, ti)
    for a, b, M in ((0, ne, Me), (ne, 2 * ne, Me), (2 * ne, 2 * ne + ni, Mi), (2 * ne + ni, p.n, Mi)):
        r = _rel(M @ z[a:b], y[a:b])
        print(f"  M z = y on [{a}, {b}): {r:.2e}")
        assert r < 1e-13
    del Me, Mi
    out, st, code = p.solve([[0.0, 0.0, 1.0]], tol=1e-6, maxit=2000)
    assert code == B.OK, st
    assert st["rel_residual"] <= 1.01e-6
    print(f"N_ext {ne} solve: {st['iterations']} steps, true residual {st['rel_residual']:.2e}")
