"""The graph partitioner of the block-wise method (cggm_partition_graph;
Sec. 4.1 clusters the graph of Lambda's active set, Sec. 4.2 the columns of
Theta through the graph of Theta^T Theta), called through the library on
the host (no GPU): the cut it reports equals a recount, part sizes respect
the bound, and on the paper's clustered graphs (Sec. 5.1) and on a Theta
with planted column groups it finds the planted structure under a random
relabelling.  A partition is not unique, so the checks are its validity and
its cut against the planted one."""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

import synth


@pytest.fixture(scope="module")
def lib():
    import os
    import paper_1509_04681_amd as m
    if not os.path.exists(m.LIB_PATH):
        from paper_1509_04681_amd import build
        build.build()
    lib = m.load()
    lib.cggm_partition_graph.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                         ctypes.c_int64, ctypes.c_double, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_int64)]
    lib.cggm_partition_graph.restype = ctypes.c_int
    return lib


def partition(lib, A, k, imbalance=0.05):
    A = sp.csr_matrix(A)
    n = A.shape[0]
    rp = np.ascontiguousarray(A.indptr, dtype=np.int64)
    col = np.ascontiguousarray(A.indices, dtype=np.int32)
    part = np.full(n, -7, dtype=np.int32)
    cut = ctypes.c_int64(-1)
    rc = lib.cggm_partition_graph(n, rp.ctypes.data, col.ctypes.data if col.size else None, k,
                                  imbalance, part.ctypes.data, ctypes.byref(cut))
    return rc, part, cut.value


def recount(A, part):
    U = sp.triu(sp.csr_matrix(A), 1).tocoo()
    L = sp.triu(sp.csr_matrix(A).T, 1).tocoo()
    pairs = set(zip(U.row.tolist(), U.col.tolist())) | set(zip(L.row.tolist(), L.col.tolist()))
    return sum(part[i] != part[j] for i, j in pairs)


def check_sizes(part, n, k, imbalance):
    sizes = np.bincount(part, minlength=k)
    cap = max(-(-n // k), int((1 + imbalance) * n / k))
    assert part.min() >= 0 and part.max() < k
    assert sizes.min() >= 1 and sizes.max() <= cap


def permuted(A, rng):
    n = A.shape[0]
    perm = rng.permutation(n)
    P = sp.csr_matrix((np.ones(n), (perm, np.arange(n))), shape=(n, n))
    return (P @ sp.csr_matrix(A) @ P.T).tocsr(), perm


@pytest.mark.parametrize("q,seed", [(2000, 0), (20000, 1)])
def test_recovers_the_clusters_of_the_clustered_graph(lib, q, seed):
    """The paper's random graph with clustering (clusters of 250, 90% of the
    edges inside them), vertices relabelled at random: one part per cluster
    with a cut within 1% of the planted clustering's."""
    rng = np.random.default_rng(seed)
    L = synth.clustered_lambda(q, rng)
    Lp, perm = permuted(L, rng)
    k = q // 250
    truth = np.empty(q, dtype=np.int32)
    truth[perm] = np.arange(q) // 250
    rc, part, cut = partition(lib, Lp, k)
    planted = recount(Lp, truth)
    print(f"clustered q={q} k={k}: cut {cut}, planted {planted}", flush=True)
    assert rc == 0
    check_sizes(part, q, k, 0.05)
    assert cut == recount(Lp, part)
    assert cut <= 1.01 * planted


def test_theta_column_blocks(lib):
    """Sec. 4.2: columns of Theta partitioned through the graph of the
    nonzeros of Theta^T Theta, so that a row's active entries fall in few
    column blocks.  Theta (p = 3000, q = 1000) whose active rows each touch
    one of 10 planted column groups (plus 3% stray entries), columns
    relabelled at random: the partition needs at most 5% more nonempty
    (row, block) pairs than the planted groups, and under half of those of
    contiguous blocks of the relabelled columns."""
    rng = np.random.default_rng(2)
    p, q, g = 3000, 1000, 10
    rows, cols = [], []
    for i in range(p):
        grp = rng.integers(g)
        c = rng.choice(np.arange(grp * 100, grp * 100 + 100), size=6, replace=False)
        rows += [i] * 6
        cols += c.tolist()
        if rng.random() < 0.03 * 6:
            rows.append(i)
            cols.append(int(rng.integers(q)))
    perm = rng.permutation(q)
    T = sp.csr_matrix((np.ones(len(rows)), (rows, perm[np.array(cols)])), shape=(p, q))
    T.data[:] = 1.0
    G = (T.T @ T).tocsr()
    rc, part, cut = partition(lib, G, g)
    assert rc == 0
    check_sizes(part, q, g, 0.05)

    def blocks(assign):
        Tc = T.tocoo()
        return len(set(zip(Tc.row.tolist(), assign[Tc.col].tolist())))

    truth = np.empty(q, dtype=np.int32)
    truth[perm] = np.arange(q) // 100
    contiguous = (np.arange(q) // 100).astype(np.int32)
    b, bt, bc = blocks(part), blocks(truth), blocks(contiguous)
    print(f"theta blocks: partition {b}, planted {bt}, contiguous {bc}", flush=True)
    assert b <= 1.05 * bt
    assert b < 0.5 * bc


def test_pattern_forms_and_determinism(lib):
    """The upper triangle alone, the full symmetric pattern and a pattern with
    repeats and self loops give the same partition; a second call repeats it."""
    rng = np.random.default_rng(3)
    A = synth.clustered_lambda(1000, rng)
    full = sp.csr_matrix(A)
    upper = sp.triu(full).tocsr()
    noisy = sp.csr_matrix(full + sp.eye(1000) + sp.triu(full, 1))
    r1 = partition(lib, full, 4)
    r2 = partition(lib, upper, 4)
    r3 = partition(lib, noisy, 4)
    r4 = partition(lib, full, 4)
    for r in (r2, r3, r4):
        assert r[0] == 0 and np.array_equal(r[1], r1[1]) and r[2] == r1[2]


def test_edge_cases(lib):
    """One part, one vertex per part, no edges, ragged sizes."""
    path = sp.diags([np.ones(36)], [1], shape=(37, 37)).tocsr()
    rc, part, cut = partition(lib, path, 1)
    assert rc == 0 and (part == 0).all() and cut == 0
    rc, part, cut = partition(lib, path, 37)
    assert rc == 0 and sorted(part.tolist()) == list(range(37)) and cut == 36
    rc, part, cut = partition(lib, path, 5, 0.0)
    assert rc == 0 and cut == 4
    check_sizes(part, 37, 5, 0.0)
    empty = sp.csr_matrix((10, 10))
    rc, part, cut = partition(lib, empty, 3, 0.0)
    assert rc == 0 and cut == 0
    check_sizes(part, 10, 3, 0.0)


def test_invalid_arguments(lib):
    import paper_1509_04681_amd as m
    rp = np.array([0, 1, 2, 2], dtype=np.int64)
    col = np.array([1, 0], dtype=np.int32)
    part = np.zeros(3, dtype=np.int32)
    cut = ctypes.c_int64()

    def call(n, rp, col, k, imb, out=part):
        return lib.cggm_partition_graph(n, rp.ctypes.data if rp is not None else None,
                                        col.ctypes.data if col is not None else None, k, imb,
                                        out.ctypes.data if out is not None else None,
                                        ctypes.byref(cut))

    assert call(3, rp, col, 2, 0.0) == m.CGGM_OK
    assert call(0, rp, col, 1, 0.0) == m.CGGM_EINVAL
    assert call(3, rp, col, 0, 0.0) == m.CGGM_EINVAL
    assert call(3, rp, col, 4, 0.0) == m.CGGM_EINVAL
    assert call(3, rp, col, 2, -0.1) == m.CGGM_EINVAL
    assert call(3, rp, col, 2, float("nan")) == m.CGGM_EINVAL
    assert call(3, None, col, 2, 0.0) == m.CGGM_EINVAL
    assert call(3, rp, None, 2, 0.0) == m.CGGM_EINVAL
    assert call(3, rp, col, 2, 0.0, out=None) == m.CGGM_EINVAL
    assert call(3, np.array([0, 2, 1, 2], dtype=np.int64), np.array([1, 0], dtype=np.int32),
                2, 0.0) == m.CGGM_EINVAL                               # decreasing rowptr
    assert call(3, rp, np.array([1, 3], dtype=np.int32), 2, 0.0) == m.CGGM_EINVAL
    assert call(3, np.array([1, 1, 2, 2], dtype=np.int64), col, 2, 0.0) == m.CGGM_EINVAL


def test_python_binding(lib):
    import paper_1509_04681_amd as m
    path = sp.diags([np.ones(99)], [1], shape=(100, 100)).tocsr()
    part, cut = m.cggm_partition_graph(path.indptr, path.indices, 4, 0.0)
    assert cut == 3 and np.array_equal(np.bincount(part), [25, 25, 25, 25])
    with pytest.raises(m.CggmError):
        m.cggm_partition_graph(path.indptr, path.indices, 101)
