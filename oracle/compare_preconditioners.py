"""FGMRES(30) iteration counts of the oracle with the block-diagonal Schur
preconditioner (eq. stoch-prec, hGS inside the Schur block, the paper's
experiments) and with hGSoc (Algorithms 2-3), on small steady problems
shaped like the solver's workloads.  Context only (test infrastructure):

    python -m oracle.compare_preconditioners

Both preconditioners use one multigrid V-cycle per A-tilde_1 solve and five
Chebyshev steps per mass solve; hGSoc is run with the third P-tilde block as
printed (A-tilde_1) and with the Schur-type reading (A-tilde_1 M^{-1} A-tilde_1).
"""
from __future__ import annotations

import sys

import numpy as np

import sg_inputs
from . import fgmres, kkt, precond

CASES = [
    # n, M, P, sigma, beta
    (16, 4, 3, 0.2, 1e-2),
    (16, 4, 3, 0.2, 1e-4),
    (32, 3, 2, 0.3, 1e-2),
    (32, 6, 2, 0.3, 1e-2),
]


def run(n, M, P, sigma, beta, max_iter=200):
    prob = kkt.Problem(n=n, M=M, P=P, sigma=sigma, beta=beta, y_target=sg_inputs.gaussian_bumps(n, 0))
    sg = kkt.setup(prob)
    b = kkt.rhs(sg)
    K = kkt.kkt_steady(sg)
    inner = precond.make_inner(sg)
    out = {}
    _, info = fgmres.fgmres(lambda v: K @ v, lambda v: precond.precond_apply(sg, v, inner), b, tol=1e-8,
                            restart=30, max_iter=max_iter)
    out["block-diagonal"] = info
    for name, adj in (("hGSoc (A-tilde_1)", "literal"), ("hGSoc (Schur reading)", "schur")):
        pt = precond.PtildeSolve(sg, "cheb", adjoint=adj)
        _, info = fgmres.fgmres(lambda v: K @ v, lambda v: precond.hgsoc(sg, v, pt, M + 1), b, tol=1e-8,
                                restart=30, max_iter=max_iter)
        out[name] = info
    return out


def main() -> int:
    print("| n | M | P | sigma | beta | block-diagonal | hGSoc (A-tilde_1) | hGSoc (Schur reading) |")
    print("|---|---|---|---|---|---|---|---|")
    for case in CASES:
        res = run(*case)
        cells = []
        for k in ("block-diagonal", "hGSoc (A-tilde_1)", "hGSoc (Schur reading)"):
            i = res[k]
            cells.append(f"{i['iters']}" if i["converged"] else f"> {i['iters']} (rel. res. {i['rel_res']:.1e})")
        print(f"| {case[0]} | {case[1]} | {case[2]} | {case[3]} | {case[4]:g} | " + " | ".join(cells) + " |",
              flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
