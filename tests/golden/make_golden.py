"""Writes lambda_table.json from the oracle's emulation of the paper's formulas.

Calls only ``oracle.paper_algorithms`` (alpha = ceil(p^(1/u)) as an exact
integer root; block size from eq. lambda-sw for (1,1) and eq. cAcB otherwise).
Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import paper_algorithms as pa  # noqa: E402

PRIMES = [1048573, 8388593, 33554393, 67108859, 2147483647, 34359738337, 68719476731,
          1099511627689, 1125899906842597, 4503599627370449]
VARIANTS = [(1, 1), (1, 2), (2, 1), (1, 3), (1, 4), (2, 2), (2, 3), (3, 2), (3, 3), (2, 4)]


def main():
    rows = []
    for p in PRIMES:
        for u, v in VARIANTS:
            rows.append({"p": p, "u": u, "v": v, "alpha": pa.iroot_ceil(p, u),
                         "beta": pa.iroot_ceil(p, v), "lambda": pa.block_size(p, u, v)})
    out = {"source": "oracle.paper_algorithms: Alg. 4 alpha, eq. lambda-sw / eq. cAcB block size, t = 53",
           "rows": rows}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lambda_table.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
