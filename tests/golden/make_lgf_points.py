"""Writes lgf_points.txt: G1 of the 7-point Laplacian (the LGF of Sec. 2.2,
L G = delta with the stencil of eq. cross_discr2) at selected lattice points,
each by adaptive quadrature of its Bessel integral (oracle.lgf_point_adaptive).
Calls only the oracle.  Run from the repository root:
    python tests/golden/make_lgf_points.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.lgf import lgf_point_adaptive  # noqa: E402

POINTS = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 0, 0), (2, 1, 0), (3, 2, 1),
          (5, 5, 5), (10, 0, 0), (17, 4, 9), (32, 32, 32), (64, 0, 0), (100, 50, 25),
          (255, 255, 255), (300, 200, 100), (512, 0, 0), (512, 512, 512)]
T_TABLE = 40.0 * 512 ** 2   # the split point the 513^3 table uses

if __name__ == "__main__":
    out = os.path.join(HERE, "lgf_points.txt")
    with open(out, "w") as fh:
        fh.write("# G1[n] of the 7-point Laplacian (paper Sec. 2.2 LGF, stencil eq. cross_discr2),\n")
        fh.write("# adaptive quadrature of -int_0^inf prod_i ive(n_i, 2t) dt, split at T = %.1f.\n" % T_TABLE)
        fh.write("# written by tests/golden/make_lgf_points.py (oracle only)\n")
        fh.write("# nx ny nz G1\n")
        for p in POINTS:
            fh.write("%d %d %d %.17e\n" % (p + (lgf_point_adaptive(p, T=T_TABLE),)))
    print("wrote", out)
