"""Oracle values for a seeded stratified subset of the batched workload
(random spheres on 32^3, 64^3 and 128^3 grids; structure recipe in
``microstructures.config_c3_structure``): C_eff from the dense basic scheme
(Alg. 1) converged to 1e-8, and the rank the converged strain needs in QTT
form.  Calls only ``oracle/``.

Rank evidence: the untruncated TT-SVD of each load case's converged strain
field (Voigt core, then the 3n bits) gives the singular values of every
bond's unfolding; truncating every bond to rank r then leaves a relative
error between max_bond sqrt(sum_{i > r} s_i^2) / ||eps|| (lower bound: one
bond alone) and sqrt(sum over bonds of the same) / ||eps|| (upper bound,
Sec. 3 eq. rounding_condition_tt).  Reported: the worst load case.

Usage: python tests/golden/make_c3_golden.py  (writes c3_subset.json)
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import microstructures as M  # noqa: E402
from oracle import dense as D  # noqa: E402

SUBSET = {5: [8, 9, 10, 11], 6: [1, 3], 7: [0]}
RANKS = [16, 32, 64, 128, 256, 512]


def bond_spectra(field, n):
    """Singular values of every bond of the untruncated TT-SVD of a
    (6, N, N, N) field in the core order Voigt, x bits, y bits, z bits."""
    T = field.reshape([6] + [2] * (3 * n))
    dims = T.shape
    M_ = T.reshape(1, -1).astype(np.complex128)
    r = 1
    spectra = []
    for k in range(len(dims) - 1):
        M_ = M_.reshape(r * dims[k], -1)
        U, s, Vh = np.linalg.svd(M_, full_matrices=False)
        keep = int(np.sum(s > s[0] * 1e-15)) if s.size else 0
        spectra.append(s)
        M_ = s[:keep, None] * Vh[:keep]
        r = keep
    return spectra


def main():
    out = []
    for n, ids in SUBSET.items():
        for i in ids:
            p = M.config_c3_structure(i)
            assert p.n == n
            C, iters, fields = D.effective_stiffness(p.phase, p.lame, p.lame0, tol=1e-8, keep_fields=True)
            lo = {r: 0.0 for r in RANKS}
            hi = {r: 0.0 for r in RANKS}
            for eps in fields:
                spectra = bond_spectra(np.asarray(eps), n)
                nrm2 = float(np.sum(np.abs(eps) ** 2))
                for r in RANKS:
                    tails = [float(np.sum(s[r:] ** 2)) for s in spectra]
                    lo[r] = max(lo[r], np.sqrt(max(tails) / nrm2))
                    hi[r] = max(hi[r], np.sqrt(sum(tails) / nrm2))
            out.append({"structure": i, "grid": 1 << n, "cap": p.cap, "spheres": p.meta["count"],
                        "E_incl": p.meta["E_incl"], "iterations": [int(v) for v in iters],
                        "ceff": np.asarray(C).reshape(-1).tolist(),
                        "rank_error_lower": {str(r): lo[r] for r in RANKS},
                        "rank_error_upper": {str(r): hi[r] for r in RANKS}})
            print(f"structure {i} ({1 << n}^3, cap {p.cap}): iterations {max(iters)}; "
                  + ", ".join(f"r{r} {lo[r]:.1e}..{hi[r]:.1e}" for r in RANKS), flush=True)
            with open(os.path.join(HERE, "c3_subset.json"), "w") as f:
                json.dump({"source": "oracle.dense.effective_stiffness(tol=1e-8), untruncated TT-SVD spectra",
                           "structures": out}, f, indent=1)


if __name__ == "__main__":
    main()
