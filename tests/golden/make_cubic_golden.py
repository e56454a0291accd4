"""Writes tests/golden/parity_cubic.json: expected values of the 3D-lattice
parity cases (open 5 x 5 x 5 boxes, the largest the oracle reaches in
seconds), computed by the oracle only: max-sum bucket elimination with the
counting tuples of Eq. (4) and traceback (Sec. III-IV), in the oracle's own
diagonal-plane order (spins sorted by x + y + z).

Inputs are not stored: each case names its seeded generator call
(instances.cubic_instances) and a SHA-256 of the coupling / field bytes.

Cases:
  * cubic5_pm1   -- 4 instances, J = +-1, h = 0: E*, g (three primes + CRT).
  * cubic5_gauss -- 4 instances, J ~ N(0,1), h ~ N(0, 0.1^2), float32: E*
                    (float64 over the float32 inputs) and the unique ground state.
Run: python tests/golden/make_cubic_golden.py   (about two minutes on 8 cores)
"""
import hashlib
import itertools
import json
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np                                    # noqa: E402

from oracle import spinglass as O                     # noqa: E402
from paper_2008_06888_amd import instances as I       # noqa: E402

OUT = os.path.join(HERE, "parity_cubic.json")
DIMS = (5, 5, 5)
BATCH = 4


def digest(inst) -> str:
    h = hashlib.sha256(np.ascontiguousarray(inst.J).tobytes())
    if inst.h is not None:
        h.update(np.ascontiguousarray(inst.h).tobytes())
    return h.hexdigest()[:16]


def diagonal_order(Lx, Ly, Lz):
    pts = sorted(itertools.product(range(Lx), range(Ly), range(Lz)), key=lambda p: (sum(p), p[2], p[1], p[0]))
    return [(z * Ly + y) * Lx + x for x, y, z in pts]


def _pm1(b):
    x = I.cubic_instances(*DIMS, batch=BATCH)[b]
    r = O.eliminate(x.n, x.edges, x.J, None, order=diagonal_order(*DIMS), counts="mod",
                    moduli=O.ORACLE_PRIMES[:4], traceback=False)
    assert r["count"] < (1 << 125)   # g <= 2^125 < the product of the four moduli
    return b, {"digest": digest(x), "energy": int(r["energy"]), "count": str(r["count"])}


def _gauss(b):
    x = I.cubic_instances(*DIMS, batch=BATCH, coupling="gauss", field_std=0.1)[b]
    r = O.eliminate(x.n, x.edges, x.J, x.h, order=diagonal_order(*DIMS))
    return b, {"digest": digest(x), "energy": float(r["energy"]),
               "sigma": "".join("1" if s < 0 else "0" for s in r["sigma"])}


def main():
    out = {"generator": "tests/golden/make_cubic_golden.py", "dims": list(DIMS)}
    with Pool(4) as pool:
        out["cubic5_pm1"] = {"cases": dict((str(b), v) for b, v in pool.map(_pm1, range(BATCH)))}
        out["cubic5_gauss"] = {"cases": dict((str(b), v) for b, v in pool.map(_gauss, range(BATCH)))}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
