"""Write the exact-arithmetic fixtures of tests/golden (calls only oracle/).

    python tests/golden/make_golden.py

Fixture rw_exact_3x3x3.txt: a 3x3x3 grid with the intensities, seeds and beta
listed in its header; the values are the exact solution of the combinatorial
Dirichlet problem (random walker, Sec. III-A of the paper) with float64 edge
weights, printed with 17 significant digits.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.exact_rational import solve_exact  # noqa: E402

SHAPE = (3, 3, 3)
# intensities: a bright centre column and a ramp, exact decimals
G = [0.1, 0.2, 0.3, 0.15, 0.8, 0.25, 0.2, 0.3, 0.4,
     0.05, 0.9, 0.2, 0.85, 0.95, 0.8, 0.1, 0.9, 0.3,
     0.2, 0.3, 0.1, 0.25, 0.75, 0.2, 0.4, 0.3, 0.2]
# label 1 at two corners, label 2 at the centre, label 3 at one face centre
LABELS = [1, 0, 0, 0, 0, 0, 0, 0, 0,
          0, 0, 0, 0, 2, 0, 0, 0, 0,
          0, 0, 0, 0, 3, 0, 0, 0, 1]
BETA = 4.0


def main():
    path = os.path.join(HERE, "rw_exact_3x3x3.txt")
    with open(path, "w") as f:
        f.write("# Exact random-walker probabilities on a 3x3x3 grid (x fastest, C order).\n")
        f.write("# Problem: combinatorial Dirichlet problem L_U x = -B^T m (Sec. III-A of the\n")
        f.write("# paper cites the random walker); weights exp(-beta (g_i - g_j)^2) in float64,\n")
        f.write("# solved exactly over the rationals by oracle/exact_rational.py.\n")
        f.write(f"# shape {SHAPE[0]} {SHAPE[1]} {SHAPE[2]}\n")
        f.write(f"# beta {BETA!r}\n")
        f.write("# g " + " ".join(repr(v) for v in G) + "\n")
        f.write("# labels " + " ".join(str(v) for v in LABELS) + "\n")
        f.write("# columns: voxel x_label1 x_label2 x_label3\n")
        xs = [solve_exact(SHAPE, G, LABELS, BETA, s) for s in (1, 2, 3)]
        for v in range(len(G)):
            f.write(f"{v} " + " ".join(f"{float(x[v]):.17g}" for x in xs) + "\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
