"""Writes tests/golden/parity_large.json: expected values of the full-size
parity cases, computed by the oracle only (max-sum bucket elimination with
the counting tuples of Eq. (4) and traceback, Sec. III-IV).

Inputs are not stored: every case names the seeded generator call that
rebuilds it, with a SHA-256 of the coupling (and field) bytes so that a
changed generator is caught instead of silently compared.

Cases:
  * square16_pm1_b64   -- 64 open 16x16 lattices, J = +-1, h = 0 (the ground-state
                          solves/s workload): E* and the exact degeneracy g.
  * square16_gauss_b64 -- 64 open 16x16 lattices, J ~ N(0,1), h ~ N(0, 0.1^2), float32:
                          E* (float64 over the float32 inputs) and the ground state.
  * reg3_uneven16      -- the 16 random 3-regular graphs (n = 100 + 20 (i mod 7)),
                          J ~ N(0,1), h = 0: E* and one ground state (unique up to a
                          global flip) for the instances whose min-fill width the
                          oracle can hold in memory.
Run: python tests/golden/make_parity_golden.py   (about a minute on 8 cores)
"""
import hashlib
import json
import os
import sys
from multiprocessing import Pool

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np                                    # noqa: E402

from oracle import spinglass as O                     # noqa: E402
from paper_2008_06888_amd import instances as I       # noqa: E402

OUT = os.path.join(HERE, "parity_large.json")
# the largest elimination table the oracle may build (2^w float64 entries)
MAX_ORACLE_WIDTH = 28


def digest(inst) -> str:
    h = hashlib.sha256(np.ascontiguousarray(inst.J).tobytes())
    if inst.h is not None:
        h.update(np.ascontiguousarray(inst.h).tobytes())
    return h.hexdigest()[:16]


def sigma_str(sigma) -> str:
    """'0' for sigma = +1, '1' for sigma = -1, spin 0 first."""
    return "".join("1" if s < 0 else "0" for s in np.asarray(sigma))


def _pm1(b):
    x = I.config_instances(0, batch=64, L=16)[b]
    r = O.eliminate(x.n, x.edges, x.J, None, order=list(range(x.n)), counts="exact", traceback=False)
    return b, {"digest": digest(x), "energy": int(r["energy"]), "count": str(r["count"])}


def _gauss(b):
    x = I.config_instances(1)[b]
    r = O.eliminate(x.n, x.edges, x.J, x.h, order=list(range(x.n)))
    return b, {"digest": digest(x), "energy": float(r["energy"]), "sigma": sigma_str(r["sigma"])}


def _reg3(i):
    x = I.config_instances(3)[i]
    order = O.min_fill_order(x.n, x.edges)
    w = O.induced_width(x.n, x.edges, order)
    if w > MAX_ORACLE_WIDTH:
        return i, {"digest": digest(x), "n": x.n, "oracle_width": w}
    r = O.eliminate(x.n, x.edges, x.J, None, order=order)
    return i, {"digest": digest(x), "n": x.n, "oracle_width": w, "energy": float(r["energy"]),
               "sigma": sigma_str(r["sigma"])}


def main():
    out = {"_source": "oracle.spinglass.eliminate (tests/golden/make_parity_golden.py)"}
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        out["square16_pm1_b64"] = {
            "generator": "instances.config_instances(0, batch=64, L=16)",
            "order": "raster", "cases": dict(sorted((str(b), v) for b, v in pool.map(_pm1, range(64))))}
        out["square16_gauss_b64"] = {
            "generator": "instances.config_instances(1)",
            "order": "raster", "cases": dict(sorted((str(b), v) for b, v in pool.map(_gauss, range(64))))}
    # widest first, one at a time: a width-28 table is 2 GiB
    reg = {}
    for i in range(16):
        k, v = _reg3(i)
        reg[str(k)] = v
        print("reg3", k, v.get("oracle_width"), v.get("energy"), flush=True)
    out["reg3_uneven16"] = {"generator": "instances.config_instances(3)", "order": "oracle min-fill",
                            "max_oracle_width": MAX_ORACLE_WIDTH, "cases": reg}
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
