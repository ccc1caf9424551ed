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
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def schedule_exe(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    exe = tmp_path_factory.mktemp("sched") / "schedule_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_1509_04681_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "schedule_test.cpp"), "-o", str(exe)],
                   check=True)
    return str(exe)


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


def sub_waves(exe, q, tile, parts):
    out = subprocess.run([exe, "dump", str(q), str(tile), str(parts)], capture_output=True,
                         text=True, check=True).stdout
    waves = []
    for line in out.splitlines():
        v = [int(x) for x in line.split()]
        waves.append([tuple(v[k:k + 4]) for k in range(0, len(v), 4)])
    return waves


def tiled_direction(Sig, Psi, G, Lam, act, lam, waves, passes):
    """Lambda CD passes run wave by wave: every tile of a sub-wave starts from
    the same D (its snapshot), runs exact Gauss-Seidel over its active upper-
    triangle coordinates in row order, and the tiles' changes are added at the
    end of the sub-wave (disjoint coordinates)."""
    q = Sig.shape[0]
    D = np.zeros((q, q))
    for _ in range(passes):
        for wave in waves:
            U = D @ Sig
            change = np.zeros((q, q))
            for r0, r1, c0, c1 in wave:
                Dl, Ul = D.copy(), U.copy()
                for i in range(r0, r1):
                    for j in range(max(i, c0), c1):
                        if not act[i, j]:
                            continue
                        if i == j:
                            a = Sig[i, i] ** 2 + 2 * Sig[i, i] * Psi[i, i]
                        else:
                            a = (Sig[i, j] ** 2 + Sig[i, i] * Sig[j, j] + Sig[i, i] * Psi[j, j]
                                 + Sig[j, j] * Psi[i, i] + 2 * Sig[i, j] * Psi[i, j])
                        b = G[i, j] + Sig[i] @ Ul[:, j] + Psi[i] @ Ul[:, j] + Psi[j] @ Ul[:, i]
                        c = Lam[i, j] + Dl[i, j]
                        w = c - b / a
                        mu = -c + np.sign(w) * max(abs(w) - lam / a, 0.0)
                        if mu == 0.0:
                            continue
                        Dl[i, j] += mu
                        Ul[i] += mu * Sig[j]
                        if i != j:
                            Dl[j, i] += mu
                            Ul[j] += mu * Sig[i]
                change += Dl - D
            D = D + change
    return D


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
