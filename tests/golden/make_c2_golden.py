"""Write tests/golden/c2_oracle.json: the CPU oracle's BiCGSTAB solve of the
128^3 workload (4 x 4 x 4 subdomains of 32^3 cells, overlap 1, eps_r U[1,10]
on 8^3-cell cubes, c = 2, right-hand side N(0,1), seed 2; right-preconditioned
BiCGSTAB in FP64 to relative residual 1e-8 from x0 = 0; Sec. IV-A).

Calls only the oracle and the seeded input generator.  Stored: the iteration
count, the true relative residual, the 2-norm of the solution and the solution
at 512 seeded slots.  Run from the repository root:
    python tests/golden/make_c2_golden.py
(about a minute on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import krylov, ras, yee  # noqa: E402
from paper_2508_07193_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_oracle.json")
N_SAMPLES = 512
SAMPLE_SEED = 1202


def solve_c2():
    P = inputs.make_problem("c2")
    n = P["nx"]
    eps_cell = yee.expand_eps(P["eps"], P["eps_block"], n, n, n)
    A = yee.assemble_A(n, n, n, P["c"], eps_cell)

    def Aop(v):
        return yee.to_padded(A @ yee.from_padded(v), n, n, n)

    def Mop(v):
        return ras.ras_apply(v, P["c"], P["sub"], 1, eps_cell)

    t0 = time.perf_counter()
    x, info = krylov.bicgstab(Aop, P["rhs"], M=Mop, tol=P["tol"], maxiter=500)
    return P, x, info, time.perf_counter() - t0


def main():
    P, x, info, secs = solve_c2()
    n = P["nx"]
    slots = np.flatnonzero(inputs.unknown_slots(n, n, n).ravel())
    pick = np.sort(np.random.default_rng(SAMPLE_SEED).choice(slots, N_SAMPLES, replace=False))
    out = dict(
        workload="128^3 Yee grid, PEC walls, 4^3 subdomains of 32^3 (overlap 1), eps_r U[1,10] "
                 "on 8^3 cubes (seed 2), c=2, RHS N(0,1); BiCGSTAB FP64 to 1e-8, x0 = 0",
        source="oracle.krylov.bicgstab with oracle.ras.ras_apply and oracle.yee.assemble_A",
        iterations=int(info["iterations"]), rel_residual_true=float(info["rel_true"]),
        converged=bool(info["converged"]), x_norm2=float(np.linalg.norm(x)),
        x_maxabs=float(np.abs(x).max()), solve_seconds=round(secs, 1),
        sample_index=[int(i) for i in pick],
        sample_value=[float(v) for v in x.ravel()[pick]])
    with open(OUT, "w") as f:
        json.dump(out, f, indent=0)
    print(f"wrote {OUT}: {info['iterations']} iterations, rel res {info['rel_true']:.3e}, "
          f"{secs:.1f} s")


if __name__ == "__main__":
    main()
