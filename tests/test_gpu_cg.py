"""Columns of Sigma = Lambda^{-1} by conjugate gradients on a sparse Lambda
(cggm_sigma_columns, Sec. 4.1) against the oracles: the dense oracle's
inverse (its own Cholesky) on random sparse Lambda, and the banded oracle's
solves on the chain Lambda at q = 40000, the output size of the block-wise
configuration."""
import time

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1509_04681_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


def csr(A):
    """CSR arrays (int64 rowptr, int32 col, float64 val) of a dense matrix's
    nonzeros, as device tensors."""
    import torch
    rows, cols = np.nonzero(A)
    rowptr = np.zeros(A.shape[0] + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return (torch.from_numpy(rowptr).cuda(), torch.from_numpy(cols.astype(np.int32)).cuda(),
            torch.from_numpy(A[rows, cols].astype(np.float64)).cuda())


def chain_csr(q, diag=2.25, off=1.0):
    """The chain precision matrix (tridiagonal: diag on the diagonal, off
    beside it) in CSR, built directly at any size."""
    import torch
    i = np.arange(q)
    r = np.concatenate([i, i[:-1], i[1:]])
    c = np.concatenate([i, i[1:], i[:-1]])
    v = np.concatenate([np.full(q, diag), np.full(q - 1, off), np.full(q - 1, off)])
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    rowptr = np.zeros(q + 1, dtype=np.int64)
    np.add.at(rowptr, r + 1, 1)
    return (torch.from_numpy(np.cumsum(rowptr)).cuda(),
            torch.from_numpy(c.astype(np.int32)).cuda(), torch.from_numpy(v).cuda())


@pytest.mark.parametrize("q,k,seed", [(300, 70, 0), (129, 64, 1), (65, 1, 2)])
def test_sigma_columns_match_oracle_inverse(cg, orc, q, k, seed):
    """Random sparse Lambda (about 3 off-diagonal entries per row, diagonally
    dominant); k columns in one or two batches of 64 (the second ragged),
    repeats included: every entry within 1e-11 of the largest of Sigma, and
    a second call bit for bit the same."""
    rng = np.random.default_rng(seed)
    Lam = synth.random_spd(q, rng, degree=3.0)
    cols = rng.integers(0, q, size=k)
    cols[0] = q - 1
    Sig = orc.inverse(Lam)
    rowptr, col, val = csr(Lam)
    r = cg.cggm_sigma_columns(rowptr, col, val, cols, tol=1e-14, max_iter=2000)
    got = r.Sigma_C.cpu().numpy()
    ref = Sig[:, cols]
    err = np.abs(got - ref).max() / np.abs(Sig).max()
    print(f"sigma_columns q={q} k={k}: iters {r.iters} resid {r.resid:.2e} err {err:.2e}",
          flush=True)
    assert r.status == cg.CGGM_OK and r.resid <= 1e-14
    assert err < 1e-11
    r2 = cg.cggm_sigma_columns(rowptr, col, val, cols, tol=1e-14, max_iter=2000)
    assert np.array_equal(r2.Sigma_C.cpu().numpy(), got)


def test_sigma_columns_chain_full_size(cg):
    """The chain Lambda at q = 40000 (diagonal 2.25, neighbours 1, the
    paper's chain graph): 64 columns, the first and last among them,
    against the banded oracle's solves; time per call and per iteration."""
    import torch
    from oracle import banded
    q = 40000
    rng = np.random.default_rng(3)
    cols = np.concatenate([[0, q - 1], rng.choice(q, size=62, replace=False)])
    rowptr, col, val = chain_csr(q)
    r = cg.cggm_sigma_columns(rowptr, col, val, cols, tol=1e-13, max_iter=1000)
    torch.cuda.synchronize()
    t = time.perf_counter()
    r = cg.cggm_sigma_columns(rowptr, col, val, cols, tol=1e-13, max_iter=1000)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    ref = banded.sigma_columns(np.full(q, 2.25), np.full(q - 1, 1.0), cols)
    got = r.Sigma_C.cpu().numpy()
    err = np.abs(got - ref).max() / np.abs(ref).max()
    nnz = 3 * q - 2
    # per iteration: the CSR arrays once; R and the previous direction read,
    # the new direction and Lambda P written by the product; X and R read and
    # written, P and Lambda P read by the update (64 columns of 8 bytes a row)
    bytes_it = 12 * nnz + 8 * (q + 1) + 10 * q * 64 * 8
    print(f"sigma_columns chain q={q} k=64: {el * 1e3:.2f} ms, {r.iters} iterations, "
          f"{el / r.iters * 1e6:.1f} us per iteration ({bytes_it * r.iters / el / 1e9:.0f} GB/s "
          f"algorithmic), resid {r.resid:.2e}, err {err:.2e}", flush=True)
    assert r.status == cg.CGGM_OK
    assert err < 1e-11


def test_sigma_columns_status_paths(cg):
    """The iteration cap returns CGGM_MAXITER with a finite result; an
    indefinite Lambda meets a curvature that is not positive (CGGM_ENOTPD);
    a CSR column outside [0, q) is rejected before any product (CGGM_EINVAL)."""
    import torch
    rng = np.random.default_rng(4)
    Lam = synth.random_spd(200, rng, degree=3.0)
    rowptr, col, val = csr(Lam)
    r = cg.cggm_sigma_columns(rowptr, col, val, [5, 17], tol=1e-14, max_iter=2)
    assert r.status == cg.CGGM_MAXITER and r.iters == 2
    assert np.isfinite(r.Sigma_C.cpu().numpy()).all() and r.resid > 1e-14
    rowptr, col, val = csr(np.diag([1.0, -1.0]))
    with pytest.raises(cg.CggmError) as ei:
        cg.cggm_sigma_columns(rowptr, col, val, [1], tol=1e-12, max_iter=50)
    assert ei.value.code == cg.CGGM_ENOTPD
    rowptr = torch.tensor([0, 1, 2], dtype=torch.int64, device="cuda")
    col = torch.tensor([0, 5], dtype=torch.int32, device="cuda")
    val = torch.tensor([1.0, 1.0], dtype=torch.float64, device="cuda")
    with pytest.raises(cg.CggmError) as ei:
        cg.cggm_sigma_columns(rowptr, col, val, [0], tol=1e-12, max_iter=50)
    assert ei.value.code == cg.CGGM_EINVAL
