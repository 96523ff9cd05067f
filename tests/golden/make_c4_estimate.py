"""Write the oracle's two-order applicability estimate (Sec. 5.2) of the
1024^3 random-sphere workload's geometry at lower orders.

Runs only ``oracle.qtt.rank_estimate`` on the workload's seeded spheres
(``microstructures.config_c4``'s centres and radii) voxelised at N = 16 ..
128, one-hot TT-SVD at the workload's delta 1e-6, and stores the largest
bond ranks in ``tests/golden/c4_estimate.json``.  Usage:

    python tests/golden/make_c4_estimate.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import qtt as Q  # noqa: E402
import microstructures as M  # noqa: E402


def main():
    rng = np.random.default_rng(0)
    cs, rs = M.random_spheres(rng, 64, 0.02, 0.08, scale_to_vf=0.15, per_sphere=True)
    out = []
    for n in (4, 5, 6, 7):
        t = time.time()
        ph = M.spheres(1 << n, cs, rs).astype(np.uint8)
        rc, rf, g = Q.rank_estimate(ph, 2, 1e-6)
        bits = 3 * n
        structural = max(min(2 * 2 ** k, 2 ** (bits - k)) for k in range(1, bits))
        out.append({"n": n, "rank_coarse": rc, "rank": rf, "growth": g,
                    "structural_max": structural, "volume_fraction": float(ph.mean()),
                    "seconds": time.time() - t})
        print(out[-1], flush=True)
    with open(os.path.join(HERE, "c4_estimate.json"), "w") as f:
        json.dump({"workload": "1024^3 64 random spheres (config_c4 centres and radii)", "delta": 1e-6,
                   "source": "oracle.qtt.rank_estimate", "orders": out}, f, indent=1)


if __name__ == "__main__":
    main()
