"""Offline autotuner of the launch schedules (run on the target GPU).

For each transform length L = 2^logL, 2^12 <= L <= 2^20, it builds a
synthetic instance with M = L/2 sizes (rank-3 kernel (i/j)^a + (j/i)^a + 2,
a = 0.45, monodisperse start), lets the library's smol_autotune time
Dormand-Prince 5(4) step attempts under the candidate variants of the three
right-hand-side kernels, and prints the chosen table.  With --write it also
rewrites csrc/schedule_table.h, which the library compiles in as its default
(rebuild afterwards).

    python -m paper_2407_16559_amd.autotune [--write] [--attempts 200] [--reps 3]
"""
import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def instance(M, a=0.45, c=2.0):
    import numpy as np
    s = np.arange(1, M + 1, dtype=np.float64)
    U = np.stack([s ** a, s ** -a, np.ones(M)])
    V = np.stack([s ** -a, s ** a, np.full(M, c)])
    n0 = np.zeros(M)
    n0[0] = 1.0
    return U, V, n0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--write", action="store_true")
    ap.add_argument("--out", default=None, help="write the table here instead of csrc/")
    ap.add_argument("--attempts", type=int, default=200)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--lo", type=int, default=12)
    ap.add_argument("--hi", type=int, default=20)
    args = ap.parse_args()
    import torch

    sys.path.insert(0, os.path.dirname(HERE))
    import paper_2407_16559_amd as smol
    dev = torch.device("cuda:0")
    rows = []
    for logL in range(args.lo, args.hi + 1):
        M = 1 << (logL - 1)
        U, V, n0 = (torch.from_numpy(x).to(dev) for x in instance(M))
        smol.set_schedule(logL, (0, 0, 0))
        sched, ms0, ms = smol.autotune(U, V, 0.005, n0, method="dp5", attempts=args.attempts,
                                       reps=args.reps)
        print(f"logL={logL} M={M}: schedule {sched}, {ms0:.4f} -> {ms:.4f} ms per attempt",
              flush=True)
        rows.append((logL, sched, ms0, ms))
        smol.release_plans()
    if args.write or args.out:
        path = args.out or os.path.join(HERE, "csrc", "schedule_table.h")
        with open(path, "w") as f:
            f.write("// Default launch schedules of FP64 plans: {log2 L, variant A, variant B,\n"
                    "// variant C} (variant encoding in sched.h).  Lengths not listed use variant\n"
                    "// 0 for every kernel.  Rows come from paper_2407_16559_amd/autotune.py run\n"
                    "// on an MI355X (DP5 step attempts, M = L/2); a row of -1 ends the table.\n"
                    "#pragma once\n"
                    "static const int k_sched_table[][4] = {\n")
            for logL, sched, ms0, ms in rows:
                f.write(f"    {{{logL}, {sched[0]}, {sched[1]}, {sched[2]}}},  "
                        f"// {ms0:.4f} -> {ms:.4f} ms per attempt\n")
            f.write("    {-1, 0, 0, 0},\n};\n")
        print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    main()
