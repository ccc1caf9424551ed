"""Penalties of the paper's synthetic workloads, chosen as in Sec. 5.1: the
pair (lambda_Lambda, lambda_Theta) on a log-spaced grid whose estimate,
solved by the oracle to the paper's stopping rule (min-norm subgradient
l1 < 0.01 (||Lambda||_1 + ||Theta||_1)), has edge counts closest to the
ground truth's, Lambda's off-diagonal edges (counted once) and Theta's
nonzeros each.  Alternating one-dimensional searches: lambda_Lambda with
lambda_Theta fixed, then lambda_Theta with lambda_Lambda fixed, twice, from
the best common lambda.  Run on reduced instances of each generator (the
noise level of the sample statistics, hence the right penalty, depends on n,
which the generators fix).  Calls only oracle/ and synth/.

    python tests/golden/choose_lambda.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

GRID = np.round(np.geomspace(0.02, 3.0, 24), 4)


def edges(Lam, Th, eps=1e-6):
    off = np.abs(Lam) > eps
    np.fill_diagonal(off, False)
    return int(off.sum() // 2), int((np.abs(Th) > eps).sum())


def choose(make):
    pr = make(0.1, 0.1)
    tL, tT = edges(pr.Lambda_true.toarray(), pr.Theta_true.toarray())
    cache = {}

    def run(lL, lT):
        if (lL, lT) not in cache:
            pr = make(lL, lT)
            r = oracle.solve(pr.X, pr.Y, lL, lT, tol=0.01, max_iter=300)
            cache[(lL, lT)] = edges(r.Lambda, r.Theta)
            print(f"  lambda_Lambda={lL:.4f} lambda_Theta={lT:.4f} edges={cache[(lL, lT)]} "
                  f"truth={(tL, tT)} iters={r.iters}", flush=True)
        return cache[(lL, lT)]

    lam = min(GRID, key=lambda g: abs(sum(run(g, g)) - tL - tT))
    lL, lT = float(lam), float(lam)
    for _ in range(2):
        lL = float(min(GRID, key=lambda g: abs(run(g, lT)[0] - tL)))
        lT = float(min(GRID, key=lambda g: abs(run(lL, g)[1] - tT)))
    return lL, lT


def main():
    oracle.build()
    cases = {
        "paper chain p=q (n=100)":
            lambda lL, lT: synth.paper_chain_problem(200, n=100, lam=lL, lam_Theta=lT),
        "paper chain p=2q (n=100)":
            lambda lL, lT: synth.paper_chain_problem(200, p=400, n=100, lam=lL, lam_Theta=lT),
        "clustered (n=200)":
            lambda lL, lT: synth.clustered_problem(500, 500, n=200, lam=lL, lam_Theta=lT),
    }
    for name, make in cases.items():
        print(name, flush=True)
        lL, lT = choose(make)
        print(f"{name}: lambda_Lambda = {lL}, lambda_Theta = {lT}", flush=True)


if __name__ == "__main__":
    main()
