"""Pins of the banded full-size oracle (``oracle/banded.py``) against the dense
oracle, which is itself pinned to closed forms, finite differences and library
routines: on small chain problems every objective and gradient entry agrees to
rounding, at tridiagonal Lambda of several conditionings and sparse Theta."""
import numpy as np
import pytest
import scipy.sparse as sp

import synth


def chain_point(q, rng, strength):
    diag = 1.0 + rng.random(q)
    off = -strength * rng.random(q - 1)
    return diag, off


def dense_lambda(diag, off):
    return np.diag(diag) + np.diag(off, 1) + np.diag(off, -1)


@pytest.mark.parametrize("p,q,n,seed,strength", [(30, 25, 40, 0, 0.45), (7, 40, 15, 1, 0.3),
                                                 (50, 12, 80, 2, 0.49)])
def test_banded_matches_dense_oracle(oracle_lib, p, q, n, seed, strength):
    from oracle import banded
    rng = np.random.default_rng(seed)
    diag, off = chain_point(q, rng, strength)
    Theta = sp.csr_matrix(synth.dense_theta(p, q, 0.1, rng))
    X = rng.standard_normal((n, p))
    Y = rng.standard_normal((n, q))
    S = oracle_lib.stats(X, Y)
    Lam = dense_lambda(diag, off)
    Th = Theta.toarray()
    lamL, lamT = 0.07, 0.03
    f_dense = oracle_lib.objective(S, Lam, Th, lamL, lamT)
    f_band = banded.objective(X, Y, diag, off, Theta, lamL, lamT)
    assert f_band == pytest.approx(f_dense, rel=1e-12, abs=1e-12)
    GL, GT, _, _ = oracle_lib.gradient(S, Lam, Th)
    lam_pairs = [(i, j) for i in range(q) for j in range(q) if (i * 7 + j * 3) % 5 == 0]
    theta_pairs = [(k, j) for k in range(p) for j in range(q) if (k * 5 + j) % 7 == 0]
    gl, gt = banded.gradient_entries(X, Y, diag, off, Theta, lam_pairs, theta_pairs)
    li, lj = np.array(lam_pairs).T
    tk, tj = np.array(theta_pairs).T
    np.testing.assert_allclose(gl, GL[li, lj], rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(gt, GT[tk, tj], rtol=1e-11, atol=1e-12)


def test_banded_objective_on_the_benchmark_generator(oracle_lib):
    """The generator's own chain Lambda and sparse Theta (shape of the benchmark
    workloads at a size the dense oracle handles)."""
    from oracle import banded
    pr = synth.chain_problem(p=60, q=45, n=70, density=0.05, lam=0.05, seed=4)
    diag = pr.Lambda_true.diagonal()
    off = pr.Lambda_true.diagonal(1)
    S = oracle_lib.stats(pr.X, pr.Y)
    f_dense = oracle_lib.objective(S, pr.Lambda_true.toarray(), pr.Theta_true.toarray(),
                                   pr.lam_Lambda, pr.lam_Theta)
    f_band = banded.objective(pr.X, pr.Y, diag, off, pr.Theta_true, pr.lam_Lambda, pr.lam_Theta)
    assert f_band == pytest.approx(f_dense, rel=1e-12)
