"""CPU emulation of the tiled Lambda direction and of its sub-wave splitting.

The GPU runs the coordinate descent of the Newton direction (Sec. 3.1,
Eq. (6)) as waves of tiles: exact Gauss-Seidel inside a tile, the tiles of a
(sub-)wave concurrently, each seeing only the direction as it stood when the
sub-wave began.  This file models that schedule in numpy -- with the wave
lists printed by the library's own host schedule code (schedule.hpp, through
tests/cpp/schedule_test.cpp) -- and shows the premise of the adaptive split:
when the tiles of a wave are strongly coupled (here Sigma has correlation 0.9
between every pair of outputs), the concurrent passes diverge and no Armijo
step exists, while running each wave as enough consecutive sub-waves gives a
descent direction the line search accepts.  The direction, its decrease and
the line search are measured with the oracle's functions.  CPU only."""
import shutil

import numpy as np
import pytest

import synth
from tiled_emulation import build_schedule_exe, sub_waves, tiled_direction


@pytest.fixture(scope="module")
def schedule_exe(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    return build_schedule_exe(tmp_path_factory.mktemp("sched"))


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


def test_split_levels_repair_a_divergent_direction(schedule_exe, orc):
    q, tile, rho, lam = 64, 4, 0.9, 0.05
    pr = synth.chain_problem(p=q, q=q, n=4 * q, density=0.01, lam=lam, seed=1)
    S = orc.stats(pr.X, pr.Y)
    Sig0 = (1 - rho) * np.eye(q) + rho * np.ones((q, q))
    Lam0 = np.linalg.inv(Sig0)
    Lam0 = (Lam0 + Lam0.T) / 2
    Th0 = np.zeros((q, q))
    GL, GT, Sig, Psi = orc.gradient(S, Lam0, Th0)
    act, _ = orc.active_sets(GL, GT, Lam0, Th0, lam, lam)
    f0 = orc.objective(S, Lam0, Th0, lam, lam)
    out = {}
    for level in range(5):                 # 16 tiles in the first wave: 2^4 = one per sub-wave
        waves = sub_waves(schedule_exe, q, tile, 2 ** level)
        assert max(len(w) for w in waves) == max(1, 16 >> level)
        D = tiled_direction(Sig, Psi, GL, Lam0, act, lam, waves, passes=4)
        delta = np.sum(GL * D) + lam * (np.abs(Lam0 + D).sum() - np.abs(Lam0).sum())
        alpha = 0.0
        if np.isfinite(delta) and delta < 0:
            _, alpha, f, _ = orc.line_search(S, Lam0, Th0, D, GL, lam, lam, f0)
        out[level] = (delta, alpha)
        print(f"level {level}: delta {delta:.3e} alpha {alpha}")
    # all 16 (then 8) tiles concurrent: the passes diverge, no Armijo step
    for level in (0, 1):
        delta, alpha = out[level]
        assert alpha == 0.0 and (not np.isfinite(delta) or abs(delta) > 1e20)
    # split far enough, the direction descends and a step is accepted
    for level in (3, 4):
        delta, alpha = out[level]
        assert delta < 0 and alpha >= 0.125
