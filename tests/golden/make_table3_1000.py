"""Writes table3_1000_oracle.txt: the oracle's exact steady-state kappa*_xx
for the 1000 x 1000 column of Table 3 (Sec. 4.2.2).

The refined checkerboard keeps 10 x 10 squares, now of 100 x 100 points
(dx = 1e-3 m, dt = 1e-5 s, tau = 1/2, eps = 0.8, nu = 2e-6 m^2/s,
G = (2, 0) m/s^2, kappa_1 = 1e-12 m^2). The field is 200-periodic in both
directions, so the 200 x 200 torus has the same unique steady state as the
1000 x 1000 one. Each ratio is solved exactly by the sparse direct solve of
the oracle's step (oracle/direct.py); this takes several minutes per ratio,
which is why the values are stored rather than recomputed by the test suite.

    python tests/golden/make_table3_1000.py [ratio ...]
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

RATIOS = (50.0, 100.0, 1000.0, 10000.0)
OUT = os.path.join(HERE, "table3_1000_oracle.txt")


def solve(ratio):
    from oracle import direct as DS
    from paper_1312_0195_amd import inputs as I
    U = I.LatticeUnits(dx=1e-3, dt=1e-5)
    field = I.checkerboard_field(1000, 10, 1e-12, ratio * 1e-12)[:200, :200].copy()
    k = DS.keff_direct(U.kappa(field), 0.5, 0.8, U.nu(2e-6), float(U.force(2.0)))
    return ratio, U.kappa_to_phys(k[0]) / 1e-12, U.kappa_to_phys(k[3]) / 1e-12


def main():
    ratios = [float(a) for a in sys.argv[1:]] or list(RATIOS)
    # one solve at a time: each holds ~5 GB and is bound by memory bandwidth
    rows = []
    for r in ratios:
        rows.append(solve(r))
        print(rows[-1], flush=True)
    with open(OUT, "w") as fh:
        fh.write("# Written by tests/golden/make_table3_1000.py from the oracle only: exact steady\n"
                 "# state (sparse direct solve) of the 200 x 200 periodic cell of the refined\n"
                 "# checkerboard of Sec. 4.2.2, Table 3 (1000 x 1000 points, squares of 100 points).\n"
                 "# Columns: kappa_2/kappa_1, kappa*_xx, kappa*_yy [1e-12 m^2]\n")
        for r, kxx, kyy in rows:
            fh.write(f"{r:g} {kxx:.10f} {kyy:.10f}\n")
    print(open(OUT).read())


if __name__ == "__main__":
    main()
