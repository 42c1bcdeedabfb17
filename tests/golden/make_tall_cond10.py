"""Write tall_cond10_100000x2000.txt: the FP64 oracle's run of Algorithm 1 on
the supplementary tall system (100000 x 2000, cond 10, blocks of 64 rows,
lambda 1e-4) to a relative residual of 1e-8 within 5000 iterations.

Calls only the oracle and the seeded generators.  Records the iteration count
at which the stop test passes, the RRN history at a few iterations, the norm
of the returned x and x at 64 fixed indices (sampled outputs for the GPU
parity test at full size).  Run from the repository root:
    python tests/golden/make_tall_cond10.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from workloads import WORKLOADS, make  # noqa: E402

NAME = "tall_cond10_100000x2000"
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), NAME + ".txt")
MARKS = (1, 10, 100, 200, 500, 1000, 2000, 3000, 4000, 5000)


def main():
    w = make(NAME)
    A, b = w["A"], w["b"]
    m, n = A.shape
    t0 = time.time()
    S = O.cosine_rowsums(A, w["block_rows"])
    _, W = O.proposal(S, n)
    ref = O.solve(A, w["block_rows"], w["lam"], b, seed=w["seed"], tol=w["tol"],
                  max_iters=w["max_iters"], W=W, record=True)
    secs = time.time() - t0
    x = ref["x"]
    idx = np.random.default_rng([w["seed"], 99]).choice(n, 64, replace=False)
    idx.sort()
    hist = ref["rrn_hist"]
    with open(OUT, "w") as f:
        f.write(f"# FP64 oracle, Algorithm 1 on {NAME} (seeded generator, cfg {WORKLOADS[NAME]['cfg']}),\n")
        f.write(f"# blocks of {w['block_rows']} rows, lambda {w['lam']}, seed {w['seed']}, "
                f"stop at RRN < {w['tol']} or {w['max_iters']} iterations.\n")
        f.write("# Written by tests/golden/make_tall_cond10.py (oracle only); "
                f"{secs:.0f} s on {O.num_threads()} threads.\n")
        f.write(f"m {m}\nn {n}\n")
        f.write(f"iters {ref['iters']}\nconverged {int(ref['converged'])}\n")
        f.write(f"rrn {float(ref['rrn'])!r}\n")
        for i in MARKS:
            if i <= len(hist):
                f.write(f"rrn_at_{i} {float(hist[i - 1])!r}\n")
        f.write(f"xnorm {float(np.linalg.norm(x))!r}\n")
        f.write("x_idx " + " ".join(str(int(i)) for i in idx) + "\n")
        f.write("x_val " + " ".join(repr(float(x[i])) for i in idx) + "\n")
        xs = w["xstar"]
        f.write(f"rel_err_xstar {float(np.linalg.norm(x - xs) / np.linalg.norm(xs))!r}\n")
    print(open(OUT).read())


if __name__ == "__main__":
    main()
