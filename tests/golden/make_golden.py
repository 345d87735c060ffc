"""Writes tests/golden/small_cases.json from the oracle only (no GPU code involved).

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import seeded_inputs as si  # noqa: E402

CASES_SYRK = [  # (n, k, p, seed)
    (5, 7, 251, 11), (6, 4, 65521, 12), (8, 8, 3, 13), (7, 9, 131071, 14), (1, 5, 251, 15),
]
CASES_HERK = [(4, 3, 65519, 21), (5, 6, 7, 22)]
PRIMES = [3, 5, 7, 11, 13, 251, 65519, 65521, 131041, 131071]


def main():
    out = {"_about": "Expected values written by this script from the oracle; inputs from seeded_inputs.",
           "syrk": [], "herk": [], "sos_minus_one": {}}
    for n, k, p, seed in CASES_SYRK:
        A = si.uniform_residues(n, k, p, seed)
        out["syrk"].append(dict(n=n, k=k, p=p, seed=seed, C=oracle.syrk_modp(A, p).tolist()))
    for n, k, p, seed in CASES_HERK:
        Ar, Ai = si.complex_residues(n, k, p, seed)
        Cr, Ci = oracle.herk_modp2(Ar, Ai, p)
        out["herk"].append(dict(n=n, k=k, p=p, seed=seed, Cre=Cr.tolist(), Cim=Ci.tolist()))
    for p in PRIMES:
        a, b, s = oracle.sos(p, -1)
        out["sos_minus_one"][str(p)] = dict(a=a, b=b, s=s)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "small_cases.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")


if __name__ == "__main__":
    main()
