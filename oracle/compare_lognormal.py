"""FGMRES iteration counts of the oracle on Section 5's own workload
(log-normal field, Hermite chaos m = 3, p = 3, gamma = 1, indicator target)
for the truncations n_tau = 1, m + 1 and n_A, with exact mean-block solves
(the paper's direct solves).  Context only (test infrastructure):

    python -m oracle.compare_lognormal           # the table of beta variations: sigma = 0.2,
                                                 # 32 x 32 elements, unrestarted, Chebyshev-5
    python -m oracle.compare_lognormal --sigma   # the tables of sigma variations at 16 x 16
                                                 # elements, beta = 1e-4: Chebyshev-5 or direct
                                                 # mass solves, unrestarted and FGMRES(30)
"""
from __future__ import annotations

import sys

import sg_inputs
from . import fgmres, kkt, precond

N, M, P, SIGMA, GAMMA = 32, 3, 3, 0.2, 1.0
BETAS = (1e-2, 1e-3, 1e-4, 1e-5)


def run(beta, max_iter=300, n=N, sigma=SIGMA, restart=None, cheb_steps=5):
    prob = kkt.Problem(n=n, M=M, P=P, sigma=sigma, beta=beta, gamma=GAMMA, y_target=sg_inputs.indicator_target(n),
                       field="lognormal")
    sg = kkt.setup(prob)
    b = kkt.rhs(sg)
    K = kkt.kkt_steady(sg)
    inner = precond.make_inner(sg, "exact")
    out = []
    for r in (1, M + 1, len(sg.G)):
        _, info = fgmres.fgmres(lambda v: K @ v, lambda v: precond.precond_apply(sg, v, inner, r, cheb_steps),
                                b, tol=1e-8, restart=restart or max_iter, max_iter=max_iter)
        out.append(info["iters"] if info["converged"] else f"> {info['iters']}")
    return out


def main() -> int:
    if "--sigma" in sys.argv[1:]:
        print("| sigma | mass solves | restart | n_tau = 1 | n_tau = m+1 | n_tau = n_A |")
        print("|---|---|---|---|---|---|")
        for sigma in (0.01, 0.1, 0.4):
            for cheb, name in ((5, "Chebyshev-5"), (0, "direct")):
                for restart in (None, 30):
                    row = run(1e-4, n=16, sigma=sigma, restart=restart, cheb_steps=cheb)
                    print(f"| {sigma:g} | {name} | {restart or 'none'} | " + " | ".join(str(v) for v in row) + " |",
                          flush=True)
        return 0
    print("| beta | n_tau = 1 | n_tau = m+1 | n_tau = n_A |")
    print("|---|---|---|---|")
    for beta in BETAS:
        print(f"| {beta:g} | " + " | ".join(str(v) for v in run(beta)) + " |", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
