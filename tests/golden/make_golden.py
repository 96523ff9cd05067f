"""Write the oracle's effective stiffness for the benchmark workloads.

Runs only the CPU oracle (dense basic scheme, Alg. 1) on the seeded inputs
of ``microstructures`` and stores C_eff (6x6, row-major) with the iteration
counts in ``tests/golden/ceff_<name>.json``.  Usage:

    python tests/golden/make_golden.py c0 c1lam c1sph c2 c0stag c2stag
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import dense as D  # noqa: E402
import microstructures as M  # noqa: E402

# name: (problem factory, tolerance, z-invariant reduction, Green scheme)
WORKLOADS = {
    "c0": (M.config_c0, 1e-12, False, "direct"),
    "c1lam": (M.config_c1_laminate, 1e-12, False, "direct"),
    "c1sph": (M.config_c1_sphere, 1e-9, False, "direct"),
    "c2": (M.config_c2, 1e-9, True, "direct"),
    # the staggered-grid Green operator of App. A, Table 3
    "c0stag": (M.config_c0, 1e-12, False, "staggered"),
    "c2stag": (M.config_c2, 1e-9, True, "staggered"),
}


def main(names):
    for name in names:
        make, tol, zred, scheme = WORKLOADS[name]
        p = make()
        t = time.time()
        # z-invariant geometries: Alg. 1 on the (N, N, 1) slice gives the same
        # iterates (only xi_z = 0 modes carry energy; pinned in
        # tests/test_oracle_scheme.py)
        phase = p.phase[:, :, :1].copy() if zred else p.phase
        C, it = D.effective_stiffness(phase, p.lame, p.lame0, tol=tol, max_iter=5000, scheme=scheme)
        out = {"workload": p.name, "n": p.n, "tol": tol, "iterations": it, "scheme": scheme,
               "lame": p.lame.tolist(), "lame0": list(p.lame0),
               "ceff": C.ravel().tolist(), "seconds": time.time() - t,
               "grid": list(phase.shape),
               "source": "oracle.dense.effective_stiffness (Alg. 1, FP64)"}
        with open(os.path.join(HERE, f"ceff_{name}.json"), "w") as f:
            json.dump(out, f, indent=1)
        print(name, it, time.time() - t, flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(WORKLOADS))
