"""Write the exact discrete multiple-traces solutions of the full-size
workloads to tests/golden/, for the GPU parity tests.

Calls only the oracle (and the seeded input generators in synth/): every
operator row by the oracle's ordered-pair quadrature, the dense mortar and
mass matrices, the plane-wave loads, the block matrix of the printed system
(Sec. 3.3) and its LU solution (oracle.solve_mtf_inplace).

  C2  sphere, exterior icosphere L4 (2,562 nodes), interior Fibonacci 2,002
      nodes; one direction; x stored as complex128.
  C3  ellipsoid (1, 0.8, 0.6), exterior icosphere L5 (10,242 nodes),
      interior Fibonacci 8,002 nodes; one direction; complex128.
  C4  the same ellipsoid with an 8,000-node interior, k 8 / 12; all 64
      directions from one factorisation; stored as complex64 (storage
      rounding 6e-8 relative, far below the 1e-5 trace tolerance).

Each result goes to mtf_<config>.npz (arrays x, dirs) with a JSON record of
the sha1 of this script, of the oracle's sources and of the generators, the
sizes and the wall times.  Memory: the C3/C4 matrix takes 21.3 GB, filled and
factorised in place.

Usage: python tests/golden/make_mtf_traces.py [C2 C3 C4]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import oracle as O  # noqa: E402

STORE = {"C2": np.complex128, "C3": np.complex128, "C4": np.complex64}


def sha1(path):
    with open(path, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()


def log(msg):
    print(time.strftime("%H:%M:%S"), msg, flush=True)


def main(names):
    srcs = {os.path.relpath(p, ROOT): sha1(p) for p in [
        os.path.abspath(__file__),
        os.path.join(ROOT, "oracle", "oracle.py"),
        os.path.join(ROOT, "oracle", "bem_oracle.c"),
        os.path.join(ROOT, "synth", "meshes.py"),
        os.path.join(ROOT, "synth", "configs.py")]}
    O.build(force=True)
    for name in names:
        c = synth.make_config(name)
        ne, ni = len(c["ext"][0]), len(c["int"][0])
        log(f"{name}: N_ext {ne}, N_int {ni}, {len(c['dirs'])} direction(s)")
        t0 = time.time()
        X = O.solve_mtf_inplace(c["ext"], c["int"], c["k_ext"], c["k_int"], c["rho_ext"], c["rho_int"],
                                c["dirs"], log=log)
        wall = time.time() - t0
        out = os.path.join(HERE, f"mtf_{name}.npz")
        np.savez(out, x=X.astype(STORE[name]), dirs=np.asarray(c["dirs"], dtype=np.float64))
        meta = dict(config=name, n_ext=ne, n_int=ni, nrhs=int(X.shape[0]),
                    k_ext=c["k_ext"], k_int=c["k_int"], rho_ext=c["rho_ext"], rho_int=c["rho_int"],
                    singular_gauss=4, stored_as=np.dtype(STORE[name]).name, wall_s=round(wall, 1),
                    threads=os.cpu_count(), sources_sha1=srcs, file_sha1=sha1(out))
        with open(os.path.join(HERE, f"mtf_{name}.json"), "w") as f:
            json.dump(meta, f, indent=1)
        log(f"{name}: wrote {out} ({wall:.0f} s)")


if __name__ == "__main__":
    main(sys.argv[1:] or ["C2", "C3", "C4"])
