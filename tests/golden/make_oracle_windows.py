"""Write the oracle trajectory windows that the GPU tests compare against.

Calls only the FP64 oracle (oracle/) and the seeded input builders
(workloads.py).  Each window is the first 16 step attempts of Dormand--Prince
5(4) with PI control (rtol 1e-6, atol 1e-12) from the monodisperse start at
M = 65536, run by the oracle's plain O(M^2 R) right-hand side:
  single_large_dp5_w16.npz    rank-3 kernel (i/j)^a + (j/i)^a + 2, a = 0.45,
                              lambda = 0.005 (the single-large instance);
  precision_rank4_dp5_w16.npz the rank-4 product kernel
                              (i^a + j^a)(i^-a + j^-a), a = 0.3, lambda = 0.02.
Each file holds the state after the window (n), the per-attempt log rows
(t, h, err, accepted, t_after) and the counters.  A whole trajectory to
t = 1e3 needs about 10^4 direct right-hand sides (hours on a host), so only
these windows are stored.

Usage: python tests/golden/make_oracle_windows.py [threads]
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402

ATTEMPTS = 16


def window(path, U, V, lam, t_end, threads):
    M = U.shape[1]
    n0 = W.monodisperse(M)
    out, st, log = oracle.integrate(U, V, lam, n0, t_end, 1e-6, 1e-12, method=oracle.DP54,
                                    max_steps=ATTEMPTS, log_cap=ATTEMPTS, threads=threads)
    assert st["status"] == oracle.EMAXSTEPS, st
    np.savez_compressed(path, n=out, log=log,
                        counts=np.array([st["n_rhs"], st["n_accept"], st["n_reject"]]),
                        t=np.array([st["t"], st["h"], st["err"]]))
    print(path, st, flush=True)


def main():
    threads = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    c = W.WORKLOADS["single-large"]
    U, V = W.brownian_rank3(c["M"], c["a"])
    window(os.path.join(HERE, "single_large_dp5_w16.npz"), U, V, c["lam"], c["t_end"], threads)
    p = W.WORKLOADS["precision"]
    U, V = W.product_rank4(p["M"], p["a"])
    window(os.path.join(HERE, "precision_rank4_dp5_w16.npz"), U, V, p["lam"], p["t_eval"],
           threads)


if __name__ == "__main__":
    main()
