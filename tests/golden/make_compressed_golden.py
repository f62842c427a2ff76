"""Write the compression-alone error at n = 40,000 for the smooth cells.

delta_c = l(Sigma~) - l(Sigma), with Sigma~ the tile-truncated covariance
(every off-diagonal nb x nb tile of the Hilbert-ordered matrix replaced by its
SVD truncated at tol, tiles above nb/2 kept exact; paper Section 2) and l from
the blocked dense oracle, for the nu = 3/2 datasets of the n = 40,000 study
(cells 3, 4, 5: beta = 0.03, 0.1, 0.3) at nb in {400, 800} and tol in
{1e-7, 1e-9}.  The acceptance bound of a float64 TLR evaluation is
max(n max(1e-8, 0.1 tol), 10 |delta_c|).  Calls only the oracle and the seeded
input generators.  Output: compressed_c2.json beside this script.

    python tests/golden/make_compressed_golden.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthetic  # noqa: E402
from oracle import blocked as OB  # noqa: E402
from oracle import ordering as OO  # noqa: E402
from oracle.likelihood import NotPositiveDefinite  # noqa: E402

OUT = os.path.join(HERE, "compressed_c2.json")


def main():
    recs = json.load(open(OUT)) if os.path.exists(OUT) else []
    done = {(r["cell"], r["nb"], r["tol"]) for r in recs}
    for cell in (3, 4, 5):
        g = json.load(open(os.path.join(HERE, f"large_c2-{cell}.json")))
        z = np.load(os.path.join(HERE, g["z_file"]))
        locs = synthetic.jittered_grid(g["m"], synthetic.seed_for(2, synthetic.SEED_LOCS, cell))
        perm = OO.reorder(locs, "hilbert")
        lo, zo = locs[perm], z[perm]
        theta = tuple(g["theta_true"])
        for nb in (400, 800):
            for tol in (1e-7, 1e-9):
                if (cell, nb, tol) in done:
                    continue
                t0 = time.time()
                try:
                    lt = OB.loglik_blocked(lo, zo, theta, b=4000, tiles=(nb, tol, nb // 2)).loglik
                except NotPositiveDefinite:
                    lt = None
                ref = g["values"][0]["loglik"]
                recs.append({"cell": cell, "theta": list(theta), "ordering": "hilbert", "nb": nb, "tol": tol,
                             "loglik_tilde": lt, "loglik": ref, "delta_c": None if lt is None else lt - ref,
                             "seconds": time.time() - t0})
                json.dump(recs, open(OUT, "w"), indent=1)
                print(f"cell {cell} nb {nb} tol {tol}: delta_c = {recs[-1]['delta_c']}", flush=True)


if __name__ == "__main__":
    main()
