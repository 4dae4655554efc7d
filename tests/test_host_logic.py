"""Host-side logic of the library, no GPU: the C ABI loads and exports every
declared symbol, mesh validation, the mortar matrix and the Gauss-Legendre
rule against the oracle / numpy, the tuning table's file, and the bench's
one-GPU guard."""
import glob
import os
import re

import numpy as np
import pytest

import synth

B = pytest.importorskip("paper_2206_00708_amd")
from paper_2206_00708_amd import _native as N  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    L = N.load()
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(bem_\w+)\s*\(", src))
    assert names, "no declarations found"
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    assert names == set(N.SIGNATURES)


def test_gauss_legendre_matches_numpy():
    for n in (1, 2, 4, 7, 16):
        x, w = B.host_gauss_legendre(n)
        xr, wr = np.polynomial.legendre.leggauss(n)
        assert np.abs(x - 0.5 * (xr + 1)).max() < 3e-15
        assert np.abs(w - 0.5 * wr).max() < 3e-15
    with pytest.raises(B.BemError):
        B.host_gauss_legendre(17)


def _bad(xyz, tri):
    with pytest.raises(B.BemError) as e:
        B.check_mesh(xyz, tri)
    return e.value.code


def test_mesh_validation():
    xyz, tri = synth.icosphere(1)
    B.check_mesh(xyz, tri)
    assert _bad(xyz, tri[1:]) == -2                               # open
    t2 = tri.copy(); t2[5] = t2[5][[0, 2, 1]]
    assert _bad(xyz, t2) == -2                                    # one flipped triangle
    assert _bad(xyz, tri[:, [0, 2, 1]]) == -2                     # inward
    assert _bad(np.vstack([xyz, [[5.0, 5, 5]]]), tri) == -2       # unused vertex
    t3 = tri.copy(); t3[0, 1] = t3[0, 0]
    assert _bad(xyz, t3) == -2                                    # repeated vertex
    t4 = tri.copy(); t4[0, 0] = len(xyz)
    assert _bad(xyz, t4) == -2                                    # index out of range
    x5 = xyz.copy(); x5[0] = np.nan
    assert _bad(x5, tri) == -2


@pytest.mark.parametrize("name", ["C1"])
def test_host_mortar_matches_oracle(orc, name):
    import scipy.sparse as sp
    c = synth.make_config(name)
    rp, col, val, dfc = B.host_mortar(c["int"], c["ext"])
    P = sp.csr_matrix((val, col, rp), shape=(len(c["int"][0]), len(c["ext"][0]))).toarray()
    Po = orc.mortar(c["int"], c["ext"])
    assert np.abs(P - Po).max() < 1e-14 * np.abs(Po).max()
    assert dfc < 1e-12
    for r in range(len(rp) - 1):
        assert np.all(np.diff(col[rp[r]:rp[r + 1]]) > 0)


def test_host_mortar_ellipsoid_and_identical(orc):
    import scipy.sparse as sp
    (xe, te), (xi, ti), _ = synth.configs.make_pair(11, 2, "fib", 0.02, (1.0, 0.8, 0.6), int_n=150)
    rp, col, val, dfc = B.host_mortar((xi, ti), (xe, te))
    P = sp.csr_matrix((val, col, rp), shape=(len(xi), len(xe))).toarray()
    Po = orc.mortar((xi, ti), (xe, te))
    assert np.abs(P - Po).max() < 1e-14 * np.abs(Po).max()
    rp, col, val, _ = B.host_mortar((xe, te), (xe, te))
    P = sp.csr_matrix((val, col, rp), shape=(len(xe), len(xe))).toarray()
    assert np.abs(P - orc.mass(xe, te)).max() < 1e-15


def test_host_mortar_mismatch_detected():
    xe, te = synth.icosphere(2)
    xi, ti = synth.icosphere(1)
    with pytest.raises(B.BemError) as e:
        B.host_mortar((xi + np.array([3.0, 0, 0]), ti), (xe, te))
    assert e.value.code == -3


def test_phase_sincos_accuracy():
    """The kernels' sin/cos against the host libm: absolute error at the
    rounding level over the whole range of phases the reduction accepts."""
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-50, 50, 200000), rng.uniform(-2000, 2000, 100000),
                        rng.uniform(-9.9e4, 9.9e4, 100000), np.arange(-64, 65) * np.pi / 4,
                        [0.0, 1e-300, 5e-324]])
    s, c = B.host_phase_sincos(x)
    assert np.abs(s - np.sin(x)).max() < 4e-16
    assert np.abs(c - np.cos(x)).max() < 4e-16
    small = np.abs(x) < 1.0
    assert np.all(np.abs(s[small] - np.sin(x[small])) <= 2.3e-16 * np.abs(np.sin(x[small])) + 1e-300)


def test_tuning_table_file(tmp_path):
    """The tuning table reads $BEMTX_TUNE_FILE once per process ("key value..."
    lines, '#' comments and malformed lines skipped); run in a child process so
    that this process's table is not the one loaded."""
    import subprocess
    import sys
    f = tmp_path / "tune.txt"
    f.write_text("# a comment\ngemm-ops:c128:e53:i52 3 2 32\nmtf-c128:e53:i52 128\nbroken\n\nmtf-c64:e29:i29 64\n")
    code = ("import sys; sys.path.insert(0, %r); import paper_2206_00708_amd as B; "
            "t = B.tune_table(); print(sorted(t.items()))" % ROOT)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300,
                         env=dict(os.environ, BEMTX_TUNE_FILE=str(f)))
    assert out.returncode == 0, out.stderr[-2000:]
    assert out.stdout.strip().splitlines()[-1] == str(sorted({"gemm-ops:c128:e53:i52": [3, 2, 32],
                                                              "mtf-c128:e53:i52": [128],
                                                              "mtf-c64:e29:i29": [64]}.items()))


def test_bench_refuses_several_gpus():
    """bench.py runs on one GPU: --gpus 2 exits with status 2 and says so,
    before touching a device."""
    import subprocess
    import sys
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=300)
    assert out.returncode == 2
    assert "one GPU" in out.stderr
