"""The sub-wave levels of the tiled sweeps on the GPU (through the C ABI).

A tiled sweep runs each wave of tiles as 2^level consecutive sub-waves (exact
Gauss-Seidel inside a tile, concurrent across the tiles of a sub-wave).  At
any fixed level the converged solve must reach the oracle's optimum (Sec. 5.1:
f* is unique; the order of coordinate descent changes the iterates, not the
limit), and the descent guards must raise the level when the concurrent
passes give no usable direction: the case built here starts from a Lambda
whose inverse has correlation 0.9 between every pair of outputs, where whole
waves of 4 x 4 tiles diverge (shown on the CPU by
tests/test_split_emulation_cpu.py).
"""
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

F_RTOL = 1e-8
SUPPORT_EPS = 1e-6


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


def load_golden(name):
    import importlib.util
    path = os.path.join(os.path.dirname(__file__), "golden", "make_golden.py")
    spec = importlib.util.spec_from_file_location("make_golden", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    if not os.path.exists(os.path.join(os.path.dirname(__file__), "golden", f"{name}.json")):
        pytest.skip(f"tests/golden/{name}.json has not been written")
    return mod.load(name)


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def check_golden(g, gold, label):
    sL = np.abs(g.Lambda.cpu().numpy()) > SUPPORT_EPS
    sT = np.abs(g.Theta.cpu().numpy()) > SUPPORT_EPS
    mL = int((~((sL == gold["support_Lambda"]) | gold["borderline_Lambda"])).sum())
    mT = int((~((sT == gold["support_Theta"]) | gold["borderline_Theta"])).sum())
    rel = abs(g.f - gold["f_star"]) / abs(gold["f_star"])
    print(f"{label}: f_gpu={g.f!r} f*={gold['f_star']!r} rel={rel:.2e} iters={g.iters} "
          f"status={g.status} support mismatches L={mL} T={mT}", flush=True)
    assert rel <= F_RTOL
    assert mL == 0 and mT == 0


@pytest.mark.parametrize("level", [1, 3, 6])
def test_fixed_levels_reach_golden_chain530(cg, level):
    gold = load_golden("chain530")
    pr = synth.workload("chain530")
    g = cg.cggm_solve(dev(pr.X), dev(pr.Y), pr.lam_Lambda, pr.lam_Theta, tol=0.0,
                      max_iter=3000, split_level=level, split_adapt=False)
    assert all((t["sweep_split"] & 255) == level and (t["sweep_split"] >> 8) == level
               for t in g.trace)
    check_golden(g, gold, f"chain530 level {level}")


@pytest.mark.parametrize("level", [1, 3])
def test_fixed_levels_reach_golden_chain2k(cg, level):
    gold = load_golden("chain2k")
    pr = synth.workload("chain2k")
    g = cg.cggm_solve(dev(pr.X), dev(pr.Y), pr.lam_Lambda, pr.lam_Theta, tol=0.0,
                      max_iter=3000, split_level=level, split_adapt=False, trace_cap=0)
    check_golden(g, gold, f"chain2k level {level}")


def correlated_start(q, rho=0.9):
    Sig0 = (1 - rho) * np.eye(q) + rho * np.ones((q, q))
    Lam0 = np.linalg.inv(Sig0)
    return (Lam0 + Lam0.T) / 2


@pytest.mark.parametrize("adapt", [True, False])
def test_guard_splits_divergent_waves(cg, orc, adapt):
    q, lam = 64, 0.05
    pr = synth.chain_problem(p=q, q=q, n=4 * q, density=0.01, lam=lam, seed=1)
    Lam0 = correlated_start(q)
    g = cg.cggm_solve(dev(pr.X), dev(pr.Y), lam, lam, tol=0.0, max_iter=3000, tile=4,
                      warm_Lambda=dev(Lam0), warm_Theta=dev(np.zeros((q, q))),
                      split_adapt=adapt)
    o = orc.solve(pr.X, pr.Y, lam, lam, tol=0.0, max_iter=20000, stall_iters=3,
                  lambda_passes=4)
    levels = [t["sweep_split"] & 255 for t in g.trace]
    print(f"adapt={adapt}: fallbacks of the first iteration {g.trace[0]['sweep_fallbacks']} "
          f"alpha {g.trace[0]['alpha']} levels {levels[:12]} f_gpu={g.f!r} f_oracle={o.f!r} "
          f"iters={g.iters} status={g.status}", flush=True)
    # the first direction (16 concurrent diagonal tiles) diverges and is redone
    assert g.trace[0]["sweep_fallbacks"] >= 1 and g.trace[0]["alpha"] > 0
    if adapt:
        assert levels[1] >= 1                     # the level was raised ...
        assert min(levels[-3:]) < max(levels)     # ... and lowered again once steps are full
    else:
        assert set(levels) == {0}
    for t in g.trace[:-1]:                        # a step is taken only along a descent
        assert t["alpha"] == 0 or t["delta"] < 0
    f = np.array([t["f"] for t in g.trace])
    assert np.all(np.diff(f) <= 1e-12 * np.abs(f[1:]))
    assert abs(g.f - o.f) <= F_RTOL * abs(o.f)
    for a, b in ((g.Lambda.cpu().numpy(), o.Lambda), (g.Theta.cpu().numpy(), o.Theta)):
        clear = ~(((np.abs(a) >= 1e-7) & (np.abs(a) <= 1e-5)) |
                  ((np.abs(b) >= 1e-7) & (np.abs(b) <= 1e-5)))
        assert np.array_equal((np.abs(a) > SUPPORT_EPS)[clear], (np.abs(b) > SUPPORT_EPS)[clear])
