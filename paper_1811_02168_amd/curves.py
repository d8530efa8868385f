"""Kernel error against order for the optimised period and for the fixed
period [-R, R] of the earlier Fourier bilateral filter (the comparison of
Sec. III, Figs. 3-4).  Host-only: both fits come from the C library.

    python -m paper_1811_02168_amd.curves      # prints a markdown table
"""
from __future__ import annotations

from . import fobf as F


def error_vs_order(R, sigmas, Ks, eps=1e9):
    """Rows of (sigma, K, E at T = R, E at the best T, best T, mean squared
    error of each over the 2R+1 samples -- the y axis of Fig. 4)."""
    rows = []
    for s in sigmas:
        for K in Ks:
            fixed = F.fit_period(R, s, K, R)
            opt = F.fit(R, s, K, eps=eps)
            rows.append({"sigma": float(s), "K": int(K), "E_fixed": fixed.E,
                         "E_opt": opt.E, "T_opt": opt.T,
                         "mse_fixed": fixed.E / (2 * R + 1),
                         "mse_opt": opt.E / (2 * R + 1)})
    return rows


def main():
    rows = error_vs_order(255, [20.0, 40.0, 60.0, 80.0], range(1, 11))
    print("| sigma | K | E, T = R | E, best T | best T |")
    print("|---|---|---|---|---|")
    for r in rows:
        print(f"| {r['sigma']:g} | {r['K']} | {r['E_fixed']:.3e} | {r['E_opt']:.3e} "
              f"| {r['T_opt']} |")


if __name__ == "__main__":
    main()
