"""Unrestarted FGMRES iteration counts of the oracle on Section 5's own
workload (log-normal field, Hermite chaos m = 3, p = 3, sigma = 0.2,
gamma = 1, indicator target, 32 x 32 elements), for the truncations
n_tau = 1, m + 1 and n_A and the beta sweep of the paper's table of beta
variations; Chebyshev-5 mass solves and exact mean-block solves (the
paper's direct solves).  Context only (test infrastructure):

    python -m oracle.compare_lognormal
"""
from __future__ import annotations

import sys

import sg_inputs
from . import fgmres, kkt, precond

N, M, P, SIGMA, GAMMA = 32, 3, 3, 0.2, 1.0
BETAS = (1e-2, 1e-3, 1e-4, 1e-5)


def run(beta, max_iter=300):
    prob = kkt.Problem(n=N, M=M, P=P, sigma=SIGMA, beta=beta, gamma=GAMMA, y_target=sg_inputs.indicator_target(N),
                       field="lognormal")
    sg = kkt.setup(prob)
    b = kkt.rhs(sg)
    K = kkt.kkt_steady(sg)
    inner = precond.make_inner(sg, "exact")
    out = []
    for r in (1, M + 1, len(sg.G)):
        _, info = fgmres.fgmres(lambda v: K @ v, lambda v: precond.precond_apply(sg, v, inner, r), b, tol=1e-8,
                                restart=max_iter, max_iter=max_iter)
        out.append(info["iters"] if info["converged"] else f"> {info['iters']}")
    return out


def main() -> int:
    print("| beta | n_tau = 1 | n_tau = m+1 | n_tau = n_A |")
    print("|---|---|---|---|")
    for beta in BETAS:
        print(f"| {beta:g} | " + " | ".join(str(v) for v in run(beta)) + " |", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
