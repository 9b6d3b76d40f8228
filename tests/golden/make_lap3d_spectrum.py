"""Write the reference low spectrum of the 64^3 Laplacian + U[0, 2] potential.

Calls only the oracle (preconditioned LOBPCG) and the seeded generators.
Output: lap3d_pot_64_lowest.txt, one "index eigenvalue residual" line per
eigenvalue.  Run from the repository root:
    python tests/golden/make_lap3d_spectrum.py   (about 15 minutes on 6 cores)
"""

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle.reference import lowest_eigenvalues_lap3d  # noqa: E402


def main(N=64, k=180):
    A = W.laplacian_3d(N, W.random_potential(N ** 3, 1002))
    vals, res = lowest_eigenvalues_lap3d(A, N, k)
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"lap3d_pot_{N}_lowest.txt")
    with open(out, "w") as f:
        f.write(f"# lowest {k} eigenvalues of the {N}^3 7-point Laplacian + U[0,2] potential (seed 1002)\n")
        f.write("# written by tests/golden/make_lap3d_spectrum.py (preconditioned LOBPCG, oracle/reference.py)\n")
        for i, (v, r) in enumerate(zip(vals, res)):
            f.write(f"{i} {v:.15e} {r:.3e}\n")
    print(out)


if __name__ == "__main__":
    main()
