"""Writes the stored expected values under tests/golden/ (calls only oracle/).

Inputs come from the seeded generators; expected values come from the oracle's
brute force (Eq. 1 minimised over every configuration) and its elimination.
Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import spinglass as O                     # noqa: E402
from paper_2008_06888_amd import instances as I       # noqa: E402


def main():
    out = {}
    # 4x4 open square lattice, J = +-1, h = 0: brute force over 2^16 states
    for b in range(4):
        inst = I.config_instances(0, batch=4)[b]
        bf = O.brute_force(inst.n, inst.edges, inst.J, inst.h)
        out[f"square4x4_pm1_{b}"] = {
            "source": "oracle.brute_force (Eq. 1 over all 2^16 configurations)",
            "J": inst.J.tolist(), "energy": bf["energy"], "count": bf["count"],
            "first_argmin_index": bf["index"]}
    # 4x4 open square lattice, Gaussian J, h ~ N(0, 0.1^2): brute force, float64
    for b in range(2):
        inst = I.config_instances(1, batch=2, L=4)[b]
        bf = O.brute_force(inst.n, inst.edges, inst.J, inst.h)
        out[f"square4x4_gauss_{b}"] = {
            "source": "oracle.brute_force (Eq. 1, float64 over fp32 inputs)",
            "energy": bf["energy"], "sigma": bf["sigma"].tolist()}
    with open(os.path.join(HERE, "small_cases.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
