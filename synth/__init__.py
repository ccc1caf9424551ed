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


# Named workloads (shapes, densities and penalties of the benchmark configurations).
WORKLOADS = {
    # p = q = 40, n = 100, 5% dense Theta, lambda = 0.1
    "chain40": dict(p=40, q=40, n=100, density=0.05, lam=0.1),
    # p = q = 2000, n = 500, 1% dense Theta, lambda = 0.05
    "chain2k": dict(p=2000, q=2000, n=500, density=0.01, lam=0.05),
    # p = q = 20000, n = 1000, 0.05% dense Theta, lambda = 0.02
    "chain20k": dict(p=20000, q=20000, n=1000, density=0.0005, lam=0.02),
    # parity case large enough (K >= 512) that tile gradient snapshots are
    # split over several workgroups
    "chain530": dict(p=530, q=515, n=100, density=0.005, lam=0.5, seed=21),
}


def workload(name: str, seed: int | None = None) -> Problem:
    kw = dict(WORKLOADS[name])
    kw["seed"] = kw.get("seed", 0) if seed is None else seed
    return chain_problem(**kw)


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
