"""Objective and sampled gradient entries at a tridiagonal Lambda, at full size.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): used by the parity
tests at the benchmark's full sizes, where the dense oracle's O(q^3) work is out
of reach.  Plain numpy / scipy, FP64, no code shared with the GPU library or
with ``cggm_oracle.c``.

At a chain (tridiagonal) Lambda every quantity of Eq. (1) and of its gradient
(Sec. 2.1) that a single entry needs costs O(q + n p) through banded solves:

  * Sigma e_j = Lambda^{-1} e_j  is one banded solve (column j of Sigma);
  * R = X Theta Sigma (n x q): column j is X (Theta sigma_j), with Theta sparse;
  * Psi = Sigma Theta^T Sxx Theta Sigma = R^T R / n, so Psi_ij = r_i . r_j / n;
  * G_Lambda = Syy - Sigma - Psi,   G_Theta = 2 Sxy + 2 Sxx Theta Sigma
                                            = 2 (X^T Y + X^T R) / n;
  * log det Lambda from the banded Cholesky factor, and
    tr(Lambda^{-1} Theta^T Sxx Theta) = ||L^{-1} (X Theta)^T||_F^2 / n
    with Lambda = L L^T.

Inputs: X (n x p), Y (n x q) as float64 arrays; the chain Lambda as its
diagonal `diag` (q) and first off-diagonal `off` (q - 1); Theta as a
scipy.sparse matrix (p x q).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse as sp


def _lower_banded(diag, off):
    ab = np.zeros((2, diag.size))
    ab[0] = diag
    ab[1, : diag.size - 1] = off
    return ab


def _sym_banded_upper(diag, off):
    """Upper-form storage of the symmetric tridiagonal matrix for solveh_banded."""
    ab = np.zeros((2, diag.size))
    ab[0, 1:] = off
    ab[1] = diag
    return ab


def sigma_columns(diag, off, cols):
    """Columns `cols` of Sigma = Lambda^{-1} (q x len(cols))."""
    q = diag.size
    E = np.zeros((q, len(cols)))
    E[np.asarray(cols), np.arange(len(cols))] = 1.0
    return scipy.linalg.solveh_banded(_sym_banded_upper(diag, off), E)


def r_columns(X, Theta, sig_cols):
    """Columns of R = X Theta Sigma for the given Sigma columns."""
    return X @ (Theta @ sig_cols)


def objective(X, Y, diag, off, Theta, lamL, lamT):
    """Eq. (1) at the chain Lambda (diag, off) and sparse Theta."""
    n = X.shape[0]
    Theta = sp.csr_matrix(Theta)
    cb = scipy.linalg.cholesky_banded(_lower_banded(diag, off), lower=True)
    logdet = 2.0 * np.sum(np.log(cb[0]))
    # tr(Syy Lambda) over the three bands
    syy_diag = np.einsum("ki,ki->i", Y, Y) / n
    syy_off = np.einsum("ki,ki->i", Y[:, :-1], Y[:, 1:]) / n
    tr_syy = float(np.dot(syy_diag, diag) + 2.0 * np.dot(syy_off, off))
    # tr(Sxy^T Theta) over the nonzeros of Theta
    coo = Theta.tocoo()
    tr_sxy = 0.0
    for s in range(0, coo.nnz, 20000):
        r, c, v = coo.row[s:s + 20000], coo.col[s:s + 20000], coo.data[s:s + 20000]
        tr_sxy += float(np.dot(np.einsum("kt,kt->t", X[:, r], Y[:, c]) / n, v))
    # tr(Lambda^{-1} Theta^T Sxx Theta) = ||L^{-1} M^T||_F^2 / n, M = X Theta
    Mt = np.ascontiguousarray((Theta.T @ X.T))                 # q x n
    Z = scipy.linalg.solve_banded((1, 0), cb, Mt)              # L^{-1} M^T
    tr_quad = float(np.sum(Z * Z)) / n
    l1 = lamL * (np.abs(diag).sum() + 2.0 * np.abs(off).sum()) + lamT * np.abs(coo.data).sum()
    return -logdet + tr_syy + 2.0 * tr_sxy + tr_quad + l1


def gradient_entries(X, Y, diag, off, Theta, lam_pairs, theta_pairs):
    """G_Lambda at the (i, j) pairs of `lam_pairs` and G_Theta at the (k, j)
    pairs of `theta_pairs` (Sec. 2.1), one entry at a time."""
    n = X.shape[0]
    Theta = sp.csr_matrix(Theta)
    lam_pairs = np.asarray(lam_pairs, dtype=np.int64).reshape(-1, 2)
    theta_pairs = np.asarray(theta_pairs, dtype=np.int64).reshape(-1, 2)
    cols = np.unique(np.concatenate([lam_pairs.ravel(), theta_pairs[:, 1]]))
    where = {int(c): t for t, c in enumerate(cols)}
    S = sigma_columns(diag, off, cols)                          # q x m
    Rc = r_columns(X, Theta, S)                                 # n x m
    gl = np.empty(len(lam_pairs))
    for t, (i, j) in enumerate(lam_pairs):
        syy = float(np.dot(Y[:, i], Y[:, j])) / n
        sig = S[i, where[int(j)]]
        psi = float(np.dot(Rc[:, where[int(i)]], Rc[:, where[int(j)]])) / n
        gl[t] = syy - sig - psi
    gt = np.empty(len(theta_pairs))
    for t, (k, j) in enumerate(theta_pairs):
        sxy = float(np.dot(X[:, k], Y[:, j])) / n
        gam = float(np.dot(X[:, k], Rc[:, where[int(j)]])) / n
        gt[t] = 2.0 * sxy + 2.0 * gam
    return gl, gt
