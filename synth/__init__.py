"""Seeded synthetic CGGM inputs (X, Y) shared by the oracle tests and the GPU path.

This module holds no arithmetic of the estimator: it only samples data from a
known conditional Gaussian graphical model so both sides can be fed the same
inputs.  The model is the one whose negative log-likelihood is the smooth part
g of the objective (paper, Sec. 2.1, Eq. (1)):

    y | x ~ N(-Lambda^{-1} Theta^T x, Lambda^{-1})

so each row of Y is  y = -x Theta Sigma + e  with  e ~ N(0, Sigma),
Sigma = Lambda^{-1}.  Sampling e uses a Cholesky factor Lambda = L L^T and
e = z L^{-T} with z standard normal.

Workload recipe (the paper's synthetic chain experiments, Sec. 5.1, with the
chain weights and densities of the benchmark configurations):
  * Lambda: chain graph, Lambda_ii = 1.25, Lambda_{i,i+1} = Lambda_{i+1,i} = -0.5
    (strictly diagonally dominant, hence positive definite);
  * Theta: exactly round(density * p * q) positions drawn uniformly without
    replacement, values s * u with s = +-1 equiprobable and u ~ U[0.5, 1];
  * X ~ N(0, I), n x p, row-major;
  * RNG: numpy.random.default_rng(seed) (PCG64), draws in the order
    positions, signs, magnitudes, X, Z.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg
import scipy.sparse as sp

CHAIN_DIAG = 1.25
CHAIN_OFF = -0.5


@dataclasses.dataclass
class Problem:
    """One synthetic CGGM problem: data plus the ground-truth parameters."""
    X: np.ndarray            # n x p, float64, C-contiguous
    Y: np.ndarray            # n x q, float64, C-contiguous
    lam_Lambda: float
    lam_Theta: float
    Lambda_true: sp.csr_matrix
    Theta_true: sp.csr_matrix
    name: str

    @property
    def n(self) -> int:
        return self.X.shape[0]

    @property
    def p(self) -> int:
        return self.X.shape[1]

    @property
    def q(self) -> int:
        return self.Y.shape[1]


def chain_lambda(q: int) -> sp.csr_matrix:
    """Chain-graph precision matrix (tridiagonal, 1.25 on the diagonal, -0.5 off it)."""
    diag = np.full(q, CHAIN_DIAG)
    off = np.full(max(q - 1, 0), CHAIN_OFF)
    return sp.diags([off, diag, off], [-1, 0, 1], format="csr", dtype=np.float64)


def sparse_theta(p: int, q: int, density: float, rng: np.random.Generator) -> sp.csr_matrix:
    """Exactly round(density*p*q) nonzeros at uniform positions, values +-U[0.5,1]."""
    k = int(round(density * p * q))
    k = min(k, p * q)
    pos = rng.choice(p * q, size=k, replace=False) if k > 0 else np.zeros(0, np.int64)
    sign = np.where(rng.random(k) < 0.5, -1.0, 1.0)
    mag = rng.uniform(0.5, 1.0, size=k)
    rows, cols = np.divmod(pos.astype(np.int64), q)
    return sp.csr_matrix((sign * mag, (rows, cols)), shape=(p, q), dtype=np.float64)


def _chain_cholesky_banded(q: int) -> np.ndarray:
    """Lower banded Cholesky factor of the chain precision (scipy banded storage)."""
    ab = np.zeros((2, q))
    ab[0, :] = CHAIN_DIAG
    ab[1, : q - 1] = CHAIN_OFF
    return scipy.linalg.cholesky_banded(ab, lower=True)


def sample_chain_xy(Theta: sp.csr_matrix, n: int, rng: np.random.Generator,
                    x_dtype=np.float64) -> tuple[np.ndarray, np.ndarray]:
    """Draw X ~ N(0,I) and Y | X from the CGGM with chain Lambda and the given Theta."""
    p, q = Theta.shape
    X = rng.standard_normal((n, p))
    if x_dtype != np.float64:
        X = X.astype(x_dtype).astype(np.float64)
    Z = rng.standard_normal((n, q))
    cb = _chain_cholesky_banded(q)                      # Lambda = L L^T, L lower bidiagonal
    M = np.asarray((sp.csr_matrix(X) @ Theta).todense()) if Theta.nnz else np.zeros((n, q))
    mean_t = scipy.linalg.cho_solve_banded((cb, True), M.T)    # Sigma (X Theta)^T, q x n
    # e^T = L^{-T} z^T  (upper bidiagonal solve with L^T)
    ut = np.zeros((2, q))
    ut[1, :] = cb[0, :]
    ut[0, 1:] = cb[1, : q - 1]
    e_t = scipy.linalg.solve_banded((0, 1), ut, Z.T)
    Y = np.ascontiguousarray((-mean_t + e_t).T)
    return np.ascontiguousarray(X), Y


def chain_problem(p: int, q: int, n: int, density: float, lam: float, seed: int = 0,
                  lam_Theta: float | None = None, x_dtype=np.float64) -> Problem:
    """Chain-Lambda CGGM problem of the given shape (the benchmark generator)."""
    rng = np.random.default_rng(seed)
    Theta = sparse_theta(p, q, density, rng)
    X, Y = sample_chain_xy(Theta, n, rng, x_dtype=x_dtype)
    lt = lam if lam_Theta is None else lam_Theta
    return Problem(X=X, Y=Y, lam_Lambda=float(lam), lam_Theta=float(lt),
                   Lambda_true=chain_lambda(q), Theta_true=Theta,
                   name=f"chain-p{p}-q{q}-n{n}-rho{density:g}-lam{lam:g}-seed{seed}")


# ---------------------------------------------------------------------------
# The paper's own synthetic workloads (Sec. 5.1).
#   * chain: Lambda_ii = 2.25, Lambda_{i,i-1} = Lambda_{i-1,i} = 1, Theta_ii = 1
#     for i < q; with p = 2q the last q inputs are irrelevant (zero rows);
#   * clustered: Lambda's graph has clusters of 250 nodes, 90% of its edges
#     join two nodes of one cluster (a cluster drawn uniformly, then two
#     distinct nodes in it), 10% two distinct nodes anywhere; 5q edges in
#     total (average degree 10), no repeats, weight 1; the diagonal is the row's
#     absolute sum plus 1 (strictly diagonally dominant, hence positive
#     definite -- the paper only asks for a positive definite Lambda).  Theta:
#     min(p, round(100 sqrt(p))) inputs drawn without replacement; each gets
#     one edge to a uniform output, then the rest of the 10q edges go to
#     uniform (selected input, output) pairs without repeats; weight 1.
#   * X ~ N(0, I) (the paper does not state the input distribution), Y | X
#     from the model (see _sample_general); RNG order: Lambda, Theta, X, noise.
# ---------------------------------------------------------------------------
def paper_chain_problem(q: int, p: int | None = None, n: int = 100, lam: float = 0.1,
                        seed: int = 0, lam_Theta: float | None = None) -> Problem:
    p = q if p is None else p
    rng = np.random.default_rng(seed)
    Lam = sp.diags([np.ones(q - 1), np.full(q, 2.25), np.ones(q - 1)], [-1, 0, 1],
                   format="csr", dtype=np.float64)
    m = min(p, q)
    Theta = sp.csr_matrix((np.ones(m), (np.arange(m), np.arange(m))), shape=(p, q))
    X, Y = _sample_general(Lam, Theta, n, rng)
    lt = lam if lam_Theta is None else lam_Theta
    return Problem(X=X, Y=Y, lam_Lambda=float(lam), lam_Theta=float(lt), Lambda_true=Lam,
                   Theta_true=Theta, name=f"paperchain-p{p}-q{q}-n{n}-lam{lam:g}-seed{seed}")


def clustered_lambda(q: int, rng: np.random.Generator, cluster: int = 250,
                     degree: float = 10.0, within: float = 0.9) -> sp.csr_matrix:
    n_edges = int(round(degree * q / 2))
    n_clusters = max(1, (q + cluster - 1) // cluster)
    edges = set()
    max_edges = q * (q - 1) // 2
    n_edges = min(n_edges, max_edges)
    while len(edges) < n_edges:
        if rng.random() < within:
            c = int(rng.integers(n_clusters))
            lo, hi = c * cluster, min(q, (c + 1) * cluster)
            if hi - lo < 2:
                continue
            i, j = rng.integers(lo, hi, 2)
        else:
            i, j = rng.integers(0, q, 2)
        if i == j:
            continue
        edges.add((int(min(i, j)), int(max(i, j))))
    e = np.array(sorted(edges), dtype=np.int64).reshape(-1, 2)
    rows = np.concatenate([e[:, 0], e[:, 1]])
    cols = np.concatenate([e[:, 1], e[:, 0]])
    A = sp.csr_matrix((np.ones(rows.size), (rows, cols)), shape=(q, q))
    diag = np.asarray(abs(A).sum(axis=1)).ravel() + 1.0
    return (A + sp.diags(diag)).tocsr()


def clustered_theta(p: int, q: int, rng: np.random.Generator) -> sp.csr_matrix:
    n_inputs = min(p, int(round(100 * np.sqrt(p))))
    inputs = rng.choice(p, size=n_inputs, replace=False)
    n_edges = min(10 * q, n_inputs * q)
    edges = set()
    for i in inputs[: min(n_inputs, n_edges)]:
        edges.add((int(i), int(rng.integers(q))))
    while len(edges) < n_edges:
        edges.add((int(inputs[rng.integers(n_inputs)]), int(rng.integers(q))))
    e = np.array(sorted(edges), dtype=np.int64).reshape(-1, 2)
    return sp.csr_matrix((np.ones(len(e)), (e[:, 0], e[:, 1])), shape=(p, q))


def clustered_problem(p: int, q: int, n: int = 200, lam: float = 0.1, seed: int = 0,
                      lam_Theta: float | None = None) -> Problem:
    rng = np.random.default_rng(seed)
    Lam = clustered_lambda(q, rng)
    Theta = clustered_theta(p, q, rng)
    X, Y = _sample_general(Lam, Theta, n, rng)
    lt = lam if lam_Theta is None else lam_Theta
    return Problem(X=X, Y=Y, lam_Lambda=float(lam), lam_Theta=float(lt), Lambda_true=Lam,
                   Theta_true=Theta, name=f"clustered-p{p}-q{q}-n{n}-lam{lam:g}-seed{seed}")


def _sample_general(Lam: sp.csr_matrix, Theta: sp.csr_matrix, n: int,
                    rng: np.random.Generator) -> tuple[np.ndarray, np.ndarray]:
    """X ~ N(0, I); Y = -X Theta Sigma + E with E ~ N(0, Sigma) drawn as
    E = W Lambda^{-1}, W = Z1 B + Z2 diag(sqrt(r)): B has one row
    sqrt(|w|) (e_i + sign(w) e_j) per edge (i < j, weight w) and r is the
    diagonal-dominance margin Lambda_ii - sum_j |Lambda_ij| >= 0, so that
    Cov(w) = B^T B + diag(r) = Lambda and Cov(e) = Lambda^{-1}.  Solves with
    Lambda by conjugate gradients; RNG order X, Z1, Z2."""
    p, q = Theta.shape
    X = rng.standard_normal((n, p))
    Lam = sp.csr_matrix(Lam)
    up = sp.triu(Lam, 1).tocoo()
    r = Lam.diagonal() - np.asarray(abs(Lam - sp.diags(Lam.diagonal())).sum(axis=1)).ravel()
    if np.any(r < -1e-12):
        raise ValueError("the sampler needs a diagonally dominant Lambda")
    ne = up.nnz
    w = np.sqrt(np.abs(up.data))
    B = sp.csr_matrix((np.concatenate([w, w * np.sign(up.data)]),
                       (np.concatenate([np.arange(ne), np.arange(ne)]),
                        np.concatenate([up.row, up.col]))), shape=(ne, q))
    Z1 = rng.standard_normal((n, ne))
    Z2 = rng.standard_normal((n, q))
    W = np.asarray((sp.csr_matrix(Z1) @ B).todense()) + Z2 * np.sqrt(np.maximum(r, 0.0))
    M = np.asarray((sp.csr_matrix(X) @ Theta).todense()) if Theta.nnz else np.zeros((n, q))
    mean_t = _spd_solve(Lam, M.T)                             # Sigma (X Theta)^T
    e_t = _spd_solve(Lam, W.T)                                # Lambda^{-1} w^T
    Y = np.ascontiguousarray((-mean_t + e_t).T)
    return np.ascontiguousarray(X), Y


def _spd_solve(A: sp.csr_matrix, Bm: np.ndarray, rtol: float = 1e-15,
               max_iter: int = 5000) -> np.ndarray:
    """A^{-1} Bm for a sparse, strictly diagonally dominant (hence SPD and
    well-conditioned) A: conjugate gradients on all columns at once, Jacobi
    preconditioned, until every column's residual is below rtol ||b||."""
    Bm = np.ascontiguousarray(Bm, dtype=np.float64)
    dinv = 1.0 / A.diagonal()
    Xs = Bm * dinv[:, None]
    R = Bm - A @ Xs
    Zr = R * dinv[:, None]
    P = Zr.copy()
    rz = np.einsum("ij,ij->j", R, Zr)
    bnorm = np.linalg.norm(Bm, axis=0)
    for _ in range(max_iter):
        if np.all(np.linalg.norm(R, axis=0) <= rtol * np.maximum(bnorm, 1e-300)):
            break
        AP = A @ P
        pap = np.einsum("ij,ij->j", P, AP)
        alpha = np.where(pap > 0, rz / np.where(pap > 0, pap, 1.0), 0.0)
        Xs += P * alpha
        R -= AP * alpha
        Zr = R * dinv[:, None]
        rz_new = np.einsum("ij,ij->j", R, Zr)
        beta = np.where(rz > 0, rz_new / np.where(rz > 0, rz, 1.0), 0.0)
        P = Zr + P * beta
        rz = rz_new
    return Xs


# Named workloads (shapes, densities and penalties of the benchmark configurations).
WORKLOADS = {
    # p = q = 40, n = 100, 5% dense Theta, lambda = 0.1
    "chain40": dict(p=40, q=40, n=100, density=0.05, lam=0.1),
    # p = q = 2000, n = 500, 1% dense Theta, lambda = 0.05
    "chain2k": dict(p=2000, q=2000, n=500, density=0.01, lam=0.05),
    # p = q = 20000, n = 1000, 0.05% dense Theta, lambda = 0.02
    "chain20k": dict(p=20000, q=20000, n=1000, density=0.0005, lam=0.02),
    # the same generator at reduced sizes with the same sample ratio n / q =
    # 0.05 (convergence study of the 20000 x 20000 configuration)
    "chain4k": dict(p=4000, q=4000, n=200, density=0.0005, lam=0.02),
    "chain8k": dict(p=8000, q=8000, n=400, density=0.0005, lam=0.02),
    # parity case large enough (K >= 512) that tile gradient snapshots are
    # split over several workgroups
    "chain530": dict(p=530, q=515, n=100, density=0.005, lam=0.5, seed=21),
    # the paper's own synthetic workloads (Sec. 5.1) at one-GPU test sizes;
    # penalties chosen by tests/golden/choose_lambda.py (estimated edge counts
    # of Lambda and of Theta closest to the truth on reduced instances, as
    # the paper chooses them)
    "paperchain2k": dict(kind="paperchain", q=2000, n=100, lam=1.9404, lam_Theta=1.5606),
    "paperchain2k_p2q": dict(kind="paperchain", q=2000, p=4000, n=100, lam=1.9404,
                             lam_Theta=1.5606),
    "clustered2k": dict(kind="clustered", p=4000, q=2000, n=200, lam=0.0478, lam_Theta=0.1767),
    # the size of the paper's active-set-versus-time experiment (Sec. 5.1)
    "clustered20k": dict(kind="clustered", p=20000, q=10000, n=200, lam=0.0478,
                         lam_Theta=0.1767),
}


def workload(name: str, seed: int | None = None) -> Problem:
    kw = dict(WORKLOADS[name])
    kw["seed"] = kw.get("seed", 0) if seed is None else seed
    kind = kw.pop("kind", "chain")
    make = {"chain": chain_problem, "paperchain": paper_chain_problem,
            "clustered": clustered_problem}[kind]
    return make(**kw)


# ---------------------------------------------------------------------------
# Request streams (batched and served solves): problems of mixed shapes.
#   * Lambda: the chain above, or a random sparse graph of mean degree 4
#     (2q uniform undirected edges without repeats, weight -0.5, diagonal =
#     the row's absolute sum + 0.25: diagonally dominant, hence positive
#     definite);
#   * Theta: exactly round(density p q) nonzeros, +-U[0.5, 1], as above;
#   * X ~ N(0, I); Y | X from the model; shapes drawn uniformly from the given
#     integer ranges; RNG order per problem: kind, p, q, n, Lambda, Theta, X,
#     noise.  Arrival times are drawn separately by the caller.
# ---------------------------------------------------------------------------
def random_sparse_lambda(q: int, rng: np.random.Generator, degree: float = 4.0,
                         weight: float = -0.5, ridge: float = 0.25) -> sp.csr_matrix:
    m = min(int(round(degree * q / 2)), q * (q - 1) // 2)
    edges = set()
    while len(edges) < m:
        i, j = rng.integers(0, q, 2)
        if i != j:
            edges.add((int(min(i, j)), int(max(i, j))))
    e = np.array(sorted(edges), dtype=np.int64).reshape(-1, 2)
    rows = np.concatenate([e[:, 0], e[:, 1]])
    cols = np.concatenate([e[:, 1], e[:, 0]])
    A = sp.csr_matrix((np.full(rows.size, weight), (rows, cols)), shape=(q, q))
    diag = np.asarray(abs(A).sum(axis=1)).ravel() + ridge
    return (A + sp.diags(diag)).tocsr()


def stream_problem(seed: int, p_range=(100, 4000), q_range=(100, 4000),
                   n_range=(200, 2000), density: float = 0.01) -> Problem:
    """One problem of a request stream (chain or random-sparse Lambda, 50/50)."""
    rng = np.random.default_rng(seed)
    kind = "chain" if rng.random() < 0.5 else "random"
    p = int(rng.integers(p_range[0], p_range[1] + 1))
    q = int(rng.integers(q_range[0], q_range[1] + 1))
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    Lam = chain_lambda(q) if kind == "chain" else random_sparse_lambda(q, rng)
    Theta = sparse_theta(p, q, density, rng)
    X, Y = _sample_general(Lam, Theta, n, rng)
    return Problem(X=X, Y=Y, lam_Lambda=0.0, lam_Theta=0.0, Lambda_true=Lam, Theta_true=Theta,
                   name=f"{kind}-p{p}-q{q}-n{n}-rho{density:g}-seed{seed}")


def penalty_path(X: np.ndarray, Y: np.ndarray, points: int = 12, ratio: float = 0.1):
    """Log-spaced penalty pairs from the smallest penalties with an all-zero
    solution off the diagonal (lam_Lambda = max off-diagonal abs(Y^T Y / n),
    lam_Theta = 2 max abs(X^T Y / n)) down to `ratio` times those."""
    n = X.shape[0]
    Syy = Y.T @ Y / n
    np.fill_diagonal(Syy, 0.0)
    lL = float(np.abs(Syy).max()) if Y.shape[1] > 1 else 1.0
    lT = float(2.0 * np.abs(X.T @ Y / n).max())
    g = np.geomspace(1.0, ratio, points)
    return lL * g, lT * g


def random_spd(q: int, rng: np.random.Generator, degree: float = 4.0,
               weight: float = -0.5, ridge: float = 0.25) -> np.ndarray:
    """Dense random sparse-pattern precision matrix: uniform random undirected edges
    with the given weight, diagonal = row abs-sum + ridge (diagonally dominant => PD)."""
    A = np.zeros((q, q))
    m = int(round(degree * q / 2))
    if q > 1 and m > 0:
        iu, ju = np.triu_indices(q, 1)
        pick = rng.choice(iu.size, size=min(m, iu.size), replace=False)
        A[iu[pick], ju[pick]] = weight
        A = A + A.T
    np.fill_diagonal(A, np.abs(A).sum(axis=1) + ridge)
    return A


def dense_theta(p: int, q: int, density: float, rng: np.random.Generator) -> np.ndarray:
    return np.asarray(sparse_theta(p, q, density, rng).todense())
