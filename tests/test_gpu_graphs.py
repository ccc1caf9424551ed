"""Captured sweeps (options.graphs): each tiled sweep's wave loop is recorded
once into a HIP graph and replayed.  The replays run the same kernels on the
same buffers in the same order, so every result must equal the eager solve
bit for bit -- over many replays with the solver's own eager work (gradients,
line search, factorizations) in between, across the parameter-buffer swaps
of the line search, across the penalties of a path, after level changes of
the adaptive split and in the mixed mode."""
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


def same(a, b):
    return (a.f == b.f and a.iters == b.iters and
            np.array_equal(a.Lambda.cpu().numpy(), b.Lambda.cpu().numpy()) and
            np.array_equal(a.Theta.cpu().numpy(), b.Theta.cpu().numpy()) and
            [t["f"] for t in a.trace] == [t["f"] for t in b.trace])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_equals_eager(cg, precision):
    pr = synth.chain_problem(p=300, q=260, n=200, density=0.02, lam=0.08, seed=41)
    X, Y = dev(pr.X), dev(pr.Y)
    kw = dict(tol=0.0, max_iter=40, stall_iters=0, precision=precision, mixed_min_q=0)
    a = cg.cggm_solve(X, Y, pr.lam_Lambda, pr.lam_Theta, **kw)
    b = cg.cggm_solve(X, Y, pr.lam_Lambda, pr.lam_Theta, graphs=True, **kw)
    assert same(a, b)


def test_graph_replay_over_a_path(cg):
    pr = synth.chain_problem(p=120, q=200, n=150, density=0.03, lam=0.1, seed=42)
    X, Y = dev(pr.X), dev(pr.Y)
    lam = [0.4, 0.2, 0.1, 0.05]
    a = cg.cggm_solve_path(X, Y, lam, lam, tol=1e-7)
    b = cg.cggm_solve_path(X, Y, lam, lam, tol=1e-7, graphs=True)
    assert all(same(x, y) for x, y in zip(a, b))


def test_graph_replay_through_split_levels(cg):
    """The strongly coupled start of the split tests: the level rises and falls,
    so several schedules are captured and replayed."""
    q = 64
    pr = synth.chain_problem(p=q, q=q, n=4 * q, density=0.01, lam=0.05, seed=1)
    Sig0 = 0.1 * np.eye(q) + 0.9 * np.ones((q, q))
    L0 = np.linalg.inv(Sig0)
    L0 = (L0 + L0.T) / 2
    kw = dict(tol=0.0, max_iter=200, tile=4, warm_Lambda=dev(L0),
              warm_Theta=dev(np.zeros((q, q))))
    a = cg.cggm_solve(dev(pr.X), dev(pr.Y), 0.05, 0.05, **kw)
    b = cg.cggm_solve(dev(pr.X), dev(pr.Y), 0.05, 0.05, graphs=True, **kw)
    assert max(t["sweep_split"] & 255 for t in a.trace) >= 1
    assert same(a, b)


def test_autotuned_tile_in_the_server(cg):
    """The tile-edge autotuner picks one of its candidates from measured times
    (the default 64 unless a smaller edge is at least 5% faster); a request
    served with that edge (graph replay on in the server) equals the plain
    path solve with the same edge bit for bit."""
    tile, ms = cg.cggm_autotune_tile(200, 300, 250, iters=2)
    print(f"autotune 300 x 250: tile {tile}, ms per iteration {ms}", flush=True)
    assert tile in (16, 32, 64) and all(np.isfinite(v) and v > 0 for v in ms.values())
    expect = 64
    for edge in (32, 16):
        if ms[edge] < 0.95 * ms[expect]:
            expect = edge
    assert tile == expect
    pr = synth.chain_problem(p=300, q=250, n=200, density=0.02, lam=0.1, seed=43)
    X, Y = dev(pr.X), dev(pr.Y)
    lam = [0.3, 0.15, 0.08]
    ref = cg.cggm_solve_path(X, Y, lam, lam, tol=1e-6, tile=tile)
    with cg.Server(slots=2, pool_bytes=1 << 30) as srv:
        info = srv.wait(srv.submit(X, Y, lam, lam, tol=1e-6, tile=tile))
    assert info["f"] == [r.f for r in ref]
    assert info["iters"] == [r.iters for r in ref]
