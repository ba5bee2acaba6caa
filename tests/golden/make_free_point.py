"""Writes free_point_8x8x8_n20_sigma2.txt from the exact rational free-field kernel.

The file holds the quantity plotted in Fig. 1a of the paper (norm of a smeared
point source on the unit gauge field at (x, y, z=0, t=0)) for an 8^3 slice,
n = 20 steps and sigma = 2 of eq. tlSmear.  Values are exact fractions from
the multinomial sum of +-2 walks in oracle/checks.py (integer arithmetic, no
floating point); the figure itself carries no numbers.

Run:  python -m tests.golden.make_free_point
"""
import os
from fractions import Fraction

from oracle.checks import free_kernel_walks_exact

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "free_point_8x8x8_n20_sigma2.txt")


def main():
    k = free_kernel_walks_exact((8, 8, 8), 20, Fraction(2))
    with open(OUT, "w") as f:
        f.write("# |psi(x,y,0,0)| of (1 + (sigma/n) Lap_two)^n applied to a point source at the origin,\n")
        f.write("# unit gauge links, 8^3 slice, n = 20, sigma = 2 (eq. tlSmear; Fig. 1a quantity).\n")
        f.write("# Exact rational values from the multinomial walk sum. Columns: x y z value\n")
        for y in range(8):
            for x in range(8):
                f.write(f"{x} {y} 0 {abs(k[(x, y, 0)])}\n")


if __name__ == "__main__":
    main()
