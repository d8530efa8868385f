"""Writes lut_table.json: the (sigma, eps) -> (K*, T*) table of the offline
step described after Algorithm 1 (Sec. II), computed by the FP64 oracle's
Algorithm 1 only.  Run from the repository root:

    python tests/golden/make_lut_table.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402

SIGMAS = [10.0, 20.0, 40.0, 80.0]
EPS = [1e-1, 1e-3, 1e-5]


def main():
    table = O.lut_build(255, SIGMAS, EPS)
    table["source"] = ("oracle.algorithm1 at every grid point, R = 255, "
                       "Tmax = 4R (tests/golden/make_lut_table.py)")
    with open(os.path.join(HERE, "lut_table.json"), "w") as fh:
        json.dump(table, fh, indent=1)
        fh.write("\n")
    print(table["K"], table["T"])


if __name__ == "__main__":
    main()
