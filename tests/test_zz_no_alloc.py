"""The allocation-free objective (cggm_objective_noalloc, static device
scratch) against the allocating cggm_objective: the same kernels on the same
inputs, so the same bits, on two calls in a row (the second with a smaller
problem, whose workspace overlays what the first left in the scratch), and a
clean CGGM_ECAPACITY for a shape whose workspace exceeds the scratch."""
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


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def point(p, q, n, seed):
    rng = np.random.default_rng(seed)
    pr = synth.chain_problem(p=p, q=q, n=n, density=0.02, lam=0.1, seed=seed)
    A = rng.standard_normal((q, q))
    Lam = A @ A.T / q + 0.5 * np.eye(q)
    Lam = (Lam + Lam.T) / 2
    Theta = synth.dense_theta(p, q, 0.2, rng)
    return [dev(a) for a in (pr.X, pr.Y, Lam, Theta)]


def test_noalloc_objective_matches_allocating(cg):
    for p, q, n, seed in ((700, 900, 800, 1), (130, 257, 70, 2)):
        X, Y, Lam, Th = point(p, q, n, seed)
        f = cg.cggm_objective(X, Y, Lam, Th, 0.07, 0.03)
        g = cg.cggm_objective_noalloc(X, Y, Lam, Th, 0.07, 0.03)
        print(f"p={p} q={q} n={n}: f={f!r} noalloc={g!r}", flush=True)
        assert g == f
    # a non positive definite Lambda is an error, as in cggm_objective
    Lbad = Lam.clone()
    Lbad[3, 3] = -1.0
    with pytest.raises(cg.CggmError) as ei:
        cg.cggm_objective_noalloc(X, Y, Lbad, Th, 0.07, 0.03)
    assert ei.value.code == cg.CGGM_ENOTPD
    # ... and the next call is unaffected
    assert cg.cggm_objective_noalloc(X, Y, Lam, Th, 0.07, 0.03) == f


def test_noalloc_rejects_shapes_beyond_the_scratch(cg):
    import torch
    n, p, q = 1000, 4, 2000            # workspace 77 MiB > 64 MiB
    X = torch.zeros((n, p), dtype=torch.float64, device="cuda:0")
    Y = torch.zeros((n, q), dtype=torch.float64, device="cuda:0")
    Lam = torch.eye(q, dtype=torch.float64, device="cuda:0")
    Th = torch.zeros((p, q), dtype=torch.float64, device="cuda:0")
    with pytest.raises(cg.CggmError) as ei:
        cg.cggm_objective_noalloc(X, Y, Lam, Th, 0.1, 0.1)
    assert ei.value.code == cg.CGGM_ECAPACITY
    assert "static scratch" in str(ei.value)
