"""Property tests of the oracle over randomly drawn small problems
(hypothesis): on every problem the objective never increases, Lambda stays
symmetric positive definite, the solve ends at the rounding floor of f (the
stall rule) or at the stopping rule and never at the iteration cap, and the
KKT conditions of Eq. (1) hold at its end, with gradients recomputed in
numpy from their definition (Eq. (3)).  Draws with n < p + q (the regime of
the larger parity workloads) converge slowly -- thousands of iterations --
but to the same KKT point, so the cap is set high and the bound holds on
every draw.  CPU only."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import synth


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build()
    return oracle


def numpy_gradient(X, Y, Lam, Theta):
    n = X.shape[0]
    Sxx, Sxy, Syy = X.T @ X / n, X.T @ Y / n, Y.T @ Y / n
    Sig = np.linalg.inv(Lam)
    Gam = Sxx @ Theta @ Sig
    return Syy - Sig - Sig @ Theta.T @ Gam, 2 * Sxy + 2 * Gam


def kkt_violation(G, P, lam):
    nz = P != 0
    v_nz = np.abs(G[nz] + lam * np.sign(P[nz]))
    v_z = np.maximum(np.abs(G[~nz]) - lam, 0)
    return max(v_nz.max(initial=0), v_z.max(initial=0))


@settings(max_examples=60, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(p=st.integers(1, 9), q=st.integers(1, 8), n=st.integers(5, 80),
       density=st.sampled_from([0.0, 0.1, 0.3]), lam=st.floats(0.02, 0.6),
       ratio=st.floats(0.3, 3.0), seed=st.integers(0, 2**31 - 1))
def test_random_problems_converge_to_kkt(orc, p, q, n, density, lam, ratio, seed):
    pr = synth.chain_problem(p=p, q=q, n=n, density=density, lam=lam, seed=seed,
                             lam_Theta=lam * ratio)
    r = orc.solve(pr.X, pr.Y, pr.lam_Lambda, pr.lam_Theta, tol=0.0, max_iter=200000,
                  stall_iters=3)
    assert r.status in (orc.ORC_OK, orc.ORC_STALLED), (r.status, r.iters)
    f = r.trace["f"][np.isfinite(r.trace["f"])]
    assert np.all(np.diff(f) <= 1e-12 * np.abs(f[1:]) + 1e-300)
    assert np.array_equal(r.Lambda, r.Lambda.T)
    assert np.linalg.eigvalsh(r.Lambda).min() > 0
    GL, GT = numpy_gradient(pr.X, pr.Y, r.Lambda, r.Theta)
    scale = max(1.0, np.abs(GL).max(), np.abs(GT).max())
    assert kkt_violation(GL, r.Lambda, pr.lam_Lambda) < 1e-7 * scale
    assert kkt_violation(GT, r.Theta, pr.lam_Theta) < 1e-7 * scale
