"""The paper's synthetic generators (Sec. 5.1) against the recipe they follow:
chain weights and the irrelevant inputs of p = 2q; for the clustered graph
the edge count (average degree 10), the share of within-cluster edges, unit
weights, positive definiteness, and Theta's selected inputs and 10q edges;
and that Y given X has the model's conditional mean and covariance."""
import numpy as np
import scipy.sparse as sp

import synth


def test_paper_chain_structure():
    pr = synth.paper_chain_problem(50, p=100, n=30, seed=1)
    L = pr.Lambda_true.toarray()
    assert np.allclose(np.diag(L), 2.25)
    assert np.allclose(np.diag(L, 1), 1.0) and np.allclose(np.diag(L, -1), 1.0)
    assert np.count_nonzero(L) == 50 + 2 * 49
    T = pr.Theta_true.toarray()
    assert T.shape == (100, 50)
    assert np.array_equal(T[:50], np.eye(50)) and not T[50:].any()   # irrelevant inputs


def test_clustered_lambda_recipe():
    q = 1000
    L = synth.clustered_lambda(q, np.random.default_rng(3))
    off = L - sp.diags(L.diagonal())
    assert (off != off.T).nnz == 0
    n_edges = off.nnz // 2
    assert n_edges == 5 * q                                    # average degree 10
    assert np.all(off.data == 1.0)
    r, c = off.nonzero()
    within = np.mean((r // 250) == (c // 250))
    # 90% drawn inside a cluster, plus the random pairs that fall inside one
    assert 0.88 < within < 0.95
    assert np.allclose(L.diagonal(), np.asarray(abs(off).sum(axis=1)).ravel() + 1.0)
    assert np.linalg.eigvalsh(L.toarray()).min() > 0.0


def test_clustered_theta_recipe():
    p, q = 400, 30
    T = synth.clustered_theta(p, q, np.random.default_rng(4))
    assert T.nnz == 10 * q and np.all(T.data == 1.0)
    rows = np.unique(T.nonzero()[0])
    assert len(rows) <= min(p, round(100 * np.sqrt(p)))
    p2 = 40000
    T2 = synth.clustered_theta(p2, 3000, np.random.default_rng(5))
    assert len(np.unique(T2.nonzero()[0])) == round(100 * np.sqrt(p2))   # every input has an edge


def test_samples_follow_the_model():
    """E[y | x] = -Sigma Theta^T x and Cov(y | x) = Sigma, by regression on a
    large sample."""
    pr = synth.clustered_problem(6, 5, n=200000, seed=7)
    Sig = np.linalg.inv(pr.Lambda_true.toarray())
    B = np.linalg.lstsq(pr.X, pr.Y, rcond=None)[0]              # p x q
    np.testing.assert_allclose(B, -pr.Theta_true.toarray() @ Sig, atol=0.01)
    res = pr.Y - pr.X @ B
    np.testing.assert_allclose(res.T @ res / pr.n, Sig, atol=0.01)


def test_stream_problems_and_penalty_path():
    """Request-stream generator: shapes in range, both Lambda kinds, diagonally
    dominant random-sparse Lambda of mean degree 4; the first point of the
    penalty path is where the optimum has Theta = 0 and a diagonal Lambda
    (checked with the oracle), later points move off it."""
    import oracle
    oracle.build()
    kinds = set()
    for seed in range(6):
        pr = synth.stream_problem(seed, p_range=(20, 40), q_range=(15, 30), n_range=(60, 90))
        assert 20 <= pr.p <= 40 and 15 <= pr.q <= 30 and 60 <= pr.n <= 90
        L = pr.Lambda_true.toarray()
        off = L - np.diag(np.diag(L))
        assert np.all(np.diag(L) > np.abs(off).sum(axis=1))
        kinds.add(pr.name.split("-")[0])
    assert kinds == {"chain", "random"}
    q = 400
    A = synth.random_sparse_lambda(q, np.random.default_rng(1)).toarray()
    assert (np.count_nonzero(A - np.diag(np.diag(A))) // 2) == 2 * q
    pr = synth.stream_problem(11, p_range=(12, 12), q_range=(8, 8), n_range=(80, 80))
    lL, lT = synth.penalty_path(pr.X, pr.Y, points=5, ratio=0.1)
    assert np.all(np.diff(lL) < 0) and abs(lL[-1] / lL[0] - 0.1) < 1e-12
    r0 = oracle.solve(pr.X, pr.Y, lL[0] * (1 + 1e-9), lT[0] * (1 + 1e-9), tol=0.0,
                      max_iter=300, stall_iters=3)
    assert np.abs(r0.Theta).max() == 0.0
    assert np.abs(r0.Lambda - np.diag(np.diag(r0.Lambda))).max() == 0.0
    r4 = oracle.solve(pr.X, pr.Y, lL[-1], lT[-1], tol=0.0, max_iter=300, stall_iters=3)
    assert np.abs(r4.Theta).max() > 0.0
