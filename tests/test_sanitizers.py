"""The host code and the oracle's C part built with AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only) and run on small meshes: the mesh
tables and their thread pool (with the assembly strips checked for the
gather's coverage at four strip sizes), the mass and mortar matrices, the
inverse-mass patch tables and the host-only C-ABI calls of the library
(tests/sanitize/host_driver.cpp; the host pass of every source, no device
code), and every exported routine of the oracle
(tests/sanitize/oracle_driver.c).  A sanitizer report or a failed check
fails the test."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2206_00708_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _write(path, xyz, tri):
    with open(path, "w") as f:
        f.write(f"{len(xyz)} {len(tri)}\n")
        np.savetxt(f, xyz, fmt="%.17g")
        np.savetxt(f, tri, fmt="%d")


@pytest.fixture(scope="module")
def meshes(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    (xe, te), (xi, ti), _ = synth.make_pair(3, 2, "fib", 0.01, (1.0, 0.8, 0.6), int_n=200)
    _write(d / "ext.txt", xe, te)
    _write(d / "int.txt", xi, ti)
    _write(d / "bad.txt", xe, te[1:])   # an open surface
    return d


def _run(cmd, cwd):
    p = subprocess.run(cmd, cwd=cwd, env=ENV, capture_output=True, text=True, timeout=600)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "Sanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_asan_ubsan(meshes):
    exe = str(meshes / "oracle_san")
    _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fopenmp", "-std=c11",
          "-D_DEFAULT_SOURCE", os.path.join(HERE, "sanitize", "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "bem_oracle.c"), "-lm", "-o", exe], meshes)
    out = _run([exe, str(meshes / "ext.txt"), str(meshes / "int.txt")], meshes)
    assert "oracle driver ok" in out


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not found")
def test_host_code_under_asan_ubsan(meshes):
    exe = str(meshes / "host_san")
    from paper_2206_00708_amd.build import SOURCES as srcs   # the library's own source list
    # the sanitizers instrument the host pass only; device code is built as usual and never run
    flags = ["-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    objs, procs = [], []
    for s in srcs:
        o = str(meshes / (s + ".o"))
        procs.append(subprocess.Popen([HIPCC, *flags, "-x", "hip", "-c", os.path.join(CSRC, s), "-o", o], cwd=meshes,
                                      stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        objs.append(o)
    for pr in procs:
        out, _ = pr.communicate(timeout=900)
        assert pr.returncode == 0, out[-4000:]
    drv = str(meshes / "host_driver.o")
    _run([HIPCC, *flags, "-x", "hip", "-c", os.path.join(HERE, "sanitize", "host_driver.cpp"), "-o", drv], meshes)
    _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          drv, *objs, "-o", exe], meshes)
    out = _run([exe, str(meshes / "int.txt"), str(meshes / "ext.txt"), str(meshes / "bad.txt")], meshes)
    assert "host driver ok" in out
