"""Writes exact_small.json: exact rational Cholesky pivots, squared factor
entries and solutions for tiny integer SPD systems.  Calls only the oracle's
exact rational routines (oracle/exact.py); run from the repository root:

    python tests/golden/make_exact_fixtures.py
"""
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle import exact  # noqa: E402


def main():
    rng = np.random.Generator(np.random.PCG64(20140517))
    cases = []
    for n in (1, 2, 3, 5, 8):
        M = rng.integers(-4, 5, size=(n, n))
        A = (M.T @ M + n * np.eye(n, dtype=np.int64)).astype(np.int64)
        b = rng.integers(-10, 11, size=n).astype(np.int64)
        Lx, D, fail = exact.ldlt(A.astype(float))
        assert fail == 0
        # squared Cholesky entries L_ij^2 = Lunit_ij^2 * D_j, with the sign of Lunit_ij
        sq = [[str(Lx[i][j] ** 2 * D[j]) for j in range(i + 1)] for i in range(n)]
        sgn = [[(1 if Lx[i][j] > 0 else -1 if Lx[i][j] < 0 else 0) for j in range(i + 1)] for i in range(n)]
        x = exact.solve(A.astype(float), b.astype(float))
        cases.append({"n": n, "A": A.tolist(), "b": b.tolist(), "L_squared": sq,
                      "L_sign": sgn, "x": [str(v) for v in x]})
    out = {"source": "exact rational arithmetic (oracle/exact.py); Cholesky of Section 3.1 and "
                     "the solve of Eq. (3) on integer SPD matrices A = M^T M + n I",
           "cases": cases}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_small.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
