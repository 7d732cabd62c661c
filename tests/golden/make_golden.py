"""Writes tests/golden/tiny_exact.json: tiny oblique-QR problems solved at 60 digits.

Calls only the oracle's brute-force routine (definition of Section 1: R is the
Cholesky factor of Z^T A Z, Q = Z R^{-1}) and the seeded generators.  Values are
stored as hex floats so that they round-trip exactly.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import exact  # noqa: E402

CASES = [  # (name, m, n, kappa_A, kappa_Z, paper case or 0 for random)
    ("random_m10_n3", 10, 3, 1e3, 1e2, 0),
    ("random_m24_n6", 24, 6, 1e6, 1e3, 0),
    ("case3_m20_n4", 20, 4, 1e8, 1e4, 3),
    ("n1_m16", 16, 1, 1e4, 1.0, 0),
]


def hexlist(x):
    return [[float(v).hex() for v in row] for row in np.atleast_2d(x)]


def main():
    out = {}
    for i, (name, m, n, ka, kz, case) in enumerate(CASES):
        rng = W.rng_for(70, i)
        if case:
            a, z, _, _ = W.paper_case(case, rng, m, n, ka, kz)
        else:
            a, _, _ = W.dense_spd(rng, m, ka)
            z = W.tall_skinny(rng, m, n, kz)
        q, r = exact.exact_oblique_qr(a, z, dps=60)
        out[name] = dict(m=m, n=n, kappa_a=ka, kappa_z=kz, case=case,
                         A=hexlist(a), Z=hexlist(z), Q=hexlist(q), R=hexlist(r),
                         source="oracle.exact.exact_oblique_qr at 60 digits")
    with open(os.path.join(HERE, "tiny_exact.json"), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
