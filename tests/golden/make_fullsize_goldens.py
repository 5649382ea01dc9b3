"""Write the oracle's converged eigenvalues for full-size workloads to tests/golden/.

Calls only the oracle (plain FP64 CPU implementation of the method) and the
seeded workload generators; nothing from the HIP library.  Each workload takes
minutes to about an hour of one CPU core and tens of GB of host memory (the
4.2M-unknown oscillator with a 68-column block needs about 40 GB).

    python tests/golden/make_fullsize_goldens.py NAME [NAME ...]

NAME is one of the keys of WORKLOADS.  The output file oracle_<NAME>.txt holds
the workload recipe, the oracle's settings, the number of corrections, the
residual history max_{j<=q} rho_j after each correction, and one line per block column: index j (1-based), Ritz value theta_j, relative residual
rho_j = ||A u_j - theta_j M u_j|| / (theta_j ||M u_j||).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import Oracle, amg  # noqa: E402
from workloads import configs  # noqa: E402

# name: (builder, recipe text, q, qe, coarse_max, tol, max_steps)
WORKLOADS = {
    # Example 1 of the paper at its finest size (Table 1): unit square,
    # h = 1/2048, interior unknowns only; q = 14 so that every ratio printed up
    # to lambda_13 / lambda_14 is covered.  Pairs (14, 15) and (16, 17) are
    # split by less than 1e-5, so the block holds 20 vectors: lambda_21 is 6%
    # above lambda_20.  Near the FP64 floor of this mesh (about 1e-9 for rho)
    # the stop rule is rho <= 2e-9.
    "ex1_square2048": (lambda: configs.square(2048, q=14), "unit square, P1, h = 1/2048 (N = 2047^2)",
                       14, 20, 512, 2e-9, 30),
    # Example 2 of the paper at its finest size (Table 2): L-shape
    # (-1,1)^2 minus (0,1)x(-1,0), h = 1/1024, no jitter, interior unknowns only
    # (N = 2047^2 - 1024^2); q = 31 so that every ratio printed up to
    # lambda_30 / lambda_31 is covered.  lambda_31 and lambda_32 are 0.1% apart,
    # so the block holds 40 vectors: it ends at a 3% gap, with lambda_41 about
    # 1.26 lambda_31.
    "ex2_lshape1024": (lambda: configs.lshape(1024, q=31), "L-shape (-1,1)^2 minus (0,1)x(-1,0), P1, h = 1/1024, "
                       "no jitter (N = 2047^2 - 1024^2)", 31, 40, 512, 2e-9, 40),
    # Example 3 of the paper at its finest size (Table 3): (-1,1)^2 with K = 1e3
    # on [0,1]^2, 1e-3 on [-1,0]^2 and 1 elsewhere, h = 1/1024, interior
    # unknowns only (N = 2047^2); q = 31 so that every ratio printed up to
    # lambda_30 / lambda_31 is covered, and a block of 40 vectors.  With the
    # contrast of 1e6, FP64 residuals stop near rho = 1e-6; the Gauss-Seidel
    # V-cycle there leaves eigenvalue errors of the order of rho (its run
    # stalled at rho = 2e-6 with errors up to 6e-7), the Chebyshev one
    # converges to that floor, so this run smooths with Chebyshev.
    "ex3_quadrants1024": (lambda: configs.quadrants(1024, q=31), "(-1,1)^2, K = 1e3 on [0,1]^2, 1e-3 on [-1,0]^2, "
                          "1 elsewhere, P1, h = 1/1024 (N = 2047^2)", 31, 40, 512, 2e-6, 80, "chebyshev"),
    # checkerboard cube, 100^3 cells (N = 970 299), q = 20 inside the 32-member low cluster
    "cube100": (lambda: configs.cube(100, q=20), "unit cube, Kuhn P1, 100^3 cells, 4x4x4 checkerboard kappa 1 / 1e3",
                20, 32, 512, 1e-10, 80),
    # oscillator -Lap + (x^2 + y^2) on (-6, 6)^2, 2047^2 interior unknowns, q = 64
    "osc2048": (lambda: configs.oscillator(2048, q=64), "oscillator on (-6,6)^2, P1, h = 12/2048 (N = 2047^2)",
                64, 68, 700, 1e-10, 80),
}


def run(name):
    make, recipe, q, qe, coarse_max, tol, max_steps = WORKLOADS[name][:7]
    smoother = WORKLOADS[name][7] if len(WORKLOADS[name]) > 7 else "gs"
    p = make()
    A = amg.csr(p["rowptr"], p["col"], p["A"], p["n"])
    M = amg.csr(p["rowptr"], p["col"], p["M"], p["n"])
    t0 = time.time()
    o = Oracle(A, M, q=q, qe=qe, coarse_max=coarse_max, coarse_min=2 * qe + 2, smoother=smoother)
    t1 = time.time()
    print("%s: N = %d, levels %s, setup %.0f s" % (name, p["n"], [L.n for L in o.levels], t1 - t0), flush=True)
    lam, U, info = o.solve(tol=tol, max_steps=max_steps, record=True)
    t2 = time.time()
    for s, (th, rho) in enumerate(info["history"]):
        print("  step %2d  max rho_j (j <= q) %.3e" % (s, rho[:q].max()), flush=True)
    rho = info["rho"]
    path = os.path.join(HERE, "oracle_%s.txt" % name)
    with open(path, "w") as f:
        f.write("# Oracle eigenvalues (plain FP64 CPU, %s V(1,1), nested start), written by\n"
                % {"gs": "Gauss-Seidel", "chebyshev": "degree-2 Chebyshev"}[smoother])
        f.write("#   python tests/golden/make_fullsize_goldens.py %s\n" % name)
        f.write("# workload: %s; N = %d; q = %d; qe = %d; coarse_max = %d\n" % (recipe, p["n"], q, qe, coarse_max))
        f.write("# levels: %s\n" % " ".join(str(L.n) for L in o.levels))
        f.write("# corrections: %d; stop rule max_{j<=q} rho_j <= %g or %d corrections; "
                "final max_{j<=q} rho_j = %.3e\n" % (info["steps"], tol, max_steps, rho[:q].max()))
        f.write("# history (corrections: max_{j<=q} rho_j): %s\n"
                % " ".join("%d:%.3e" % (k, h[1][:q].max()) for k, h in enumerate(info["history"])))
        f.write("# j theta_j rho_j\n")
        for j in range(qe):
            f.write("%d %.17e %.3e\n" % (j + 1, lam[j], rho[j]))
    print("%s: %d corrections, %.0f s; wrote %s" % (name, info["steps"], t2 - t1, path), flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:]:
        run(n)
