"""Pins of the CPU oracle against facts the paper and the mathematics fix.

Nothing here compares the oracle with itself: every expected value comes from a
closed form, a library routine solving the same problem (sklearn lasso /
graphical lasso, scipy's Gaussian log-density), a brute-force enumeration, an
independent first-order solver, finite differences of the objective, or an
invariant of the problem (KKT, convexity, symmetry, scaling).
"""
import itertools

import numpy as np
import pytest
import scipy.stats

import synth

pytestmark = pytest.mark.filterwarnings("ignore::sklearn.exceptions.ConvergenceWarning")


def random_problem(p, q, n, seed, theta_density=0.3, noise=1.0):
    rng = np.random.default_rng(seed)
    Lam = synth.random_spd(q, rng, degree=2.0)
    Theta = synth.dense_theta(p, q, theta_density, rng)
    X = rng.standard_normal((n, p))
    Sig = np.linalg.inv(Lam)
    E = rng.multivariate_normal(np.zeros(q), Sig, size=n) * noise
    Y = -X @ Theta @ Sig + E
    return np.ascontiguousarray(X), np.ascontiguousarray(Y)


def random_state(p, q, rng):
    """A positive definite Lambda and a sparse Theta to evaluate derivatives at."""
    Lam = synth.random_spd(q, rng, degree=2.0)
    Lam = Lam + 0.3 * np.diag(rng.random(q))
    Theta = synth.dense_theta(p, q, 0.5, rng)
    return Lam, Theta


# ----------------------------------------------------------------------------
# Objective: g is twice the average Gaussian negative log-likelihood of
# y | x ~ N(-Sigma Theta^T x, Sigma), up to the constant q log(2 pi).
# ----------------------------------------------------------------------------
def test_objective_is_gaussian_nll(oracle_lib):
    o = oracle_lib
    rng = np.random.default_rng(1)
    X, Y = random_problem(5, 4, 30, seed=2)
    Lam, Theta = random_state(5, 4, rng)
    S = o.stats(X, Y)
    Sig = np.linalg.inv(Lam)
    nll = 0.0
    for k in range(X.shape[0]):
        mean = -Sig @ Theta.T @ X[k]
        nll -= scipy.stats.multivariate_normal(mean, Sig).logpdf(Y[k])
    g_expected = 2.0 * nll / X.shape[0] - 4 * np.log(2 * np.pi)
    lamL, lamT = 0.07, 0.11
    pen = lamL * np.abs(Lam).sum() + lamT * np.abs(Theta).sum()
    f = o.objective(S, Lam, Theta, lamL, lamT)
    assert f == pytest.approx(g_expected + pen, rel=1e-12, abs=1e-12)


def test_objective_not_pd_is_rejected(oracle_lib):
    o = oracle_lib
    X, Y = random_problem(3, 3, 20, seed=3)
    S = o.stats(X, Y)
    Lam = np.eye(3)
    Lam[0, 0] = -0.5
    assert o.objective(S, Lam, np.zeros((3, 3)), 0.1, 0.1) is None
    assert o.cholesky(Lam) is None


def test_stats_match_definition(oracle_lib):
    X, Y = random_problem(6, 5, 17, seed=4)
    Sxx, Sxy, Syy = oracle_lib.stats(X, Y)
    np.testing.assert_allclose(Sxx, np.cov(X.T, bias=True, ddof=0) + np.outer(X.mean(0), X.mean(0)),
                               rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(Sxy, X.T @ Y / 17, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(Syy, Y.T @ Y / 17, rtol=1e-12, atol=1e-13)


def test_cholesky_and_inverse_match_lapack(oracle_lib):
    rng = np.random.default_rng(5)
    A = synth.random_spd(9, rng, degree=3.0)
    np.testing.assert_allclose(oracle_lib.cholesky(A), np.linalg.cholesky(A), rtol=1e-13,
                               atol=1e-14)
    np.testing.assert_allclose(oracle_lib.inverse(A), np.linalg.inv(A), rtol=1e-12, atol=1e-13)


# ----------------------------------------------------------------------------
# Eq. (3) and Eq. (4) against finite differences of f (lambda = 0).
# ----------------------------------------------------------------------------
def _g(o, S, Lam, Theta):
    return o.objective(S, Lam, Theta, 0.0, 0.0)


def test_gradient_matches_finite_differences(oracle_lib):
    o = oracle_lib
    rng = np.random.default_rng(6)
    p, q = 4, 5
    X, Y = random_problem(p, q, 25, seed=7)
    S = o.stats(X, Y)
    Lam, Theta = random_state(p, q, rng)
    GL, GT, _, _ = o.gradient(S, Lam, Theta)
    eps = 1e-6
    for i in range(q):
        for j in range(q):
            E = np.zeros((q, q))
            E[i, j] = E[j, i] = 1.0
            d = (_g(o, S, Lam + eps * E, Theta) - _g(o, S, Lam - eps * E, Theta)) / (2 * eps)
            expect = GL[i, j] * (1.0 if i == j else 2.0)   # symmetric move hits (i,j) and (j,i)
            assert d == pytest.approx(expect, rel=1e-6, abs=1e-7), (i, j)
    for i in range(p):
        for j in range(q):
            E = np.zeros((p, q))
            E[i, j] = 1.0
            d = (_g(o, S, Lam, Theta + eps * E) - _g(o, S, Lam, Theta - eps * E)) / (2 * eps)
            assert d == pytest.approx(GT[i, j], rel=1e-6, abs=1e-7), (i, j)


def test_lambda_hessian_matches_finite_differences(oracle_lib):
    """Second directional derivative of g along symmetric E equals
    vec(E)^T [Sigma (x) (Sigma + 2 Psi)] vec(E) (Eq. (4))."""
    o = oracle_lib
    rng = np.random.default_rng(8)
    p, q = 3, 4
    X, Y = random_problem(p, q, 20, seed=9)
    S = o.stats(X, Y)
    Lam, Theta = random_state(p, q, rng)
    _, _, Sig, Psi = o.gradient(S, Lam, Theta)
    eps = 1e-4
    for _ in range(5):
        E = rng.standard_normal((q, q))
        E = E + E.T
        g0 = _g(o, S, Lam, Theta)
        d2 = (_g(o, S, Lam + eps * E, Theta) - 2 * g0 + _g(o, S, Lam - eps * E, Theta)) / eps**2
        e = E.reshape(-1)
        H = np.kron(Sig, Sig + 2 * Psi)
        assert d2 == pytest.approx(e @ H @ e, rel=1e-5)


# ----------------------------------------------------------------------------
# Each coordinate step is the exact 1-D minimiser of the l1-penalised model.
# The model along a coordinate is rebuilt from finite differences of f, and
# minimised by enumerating the candidate points of a convex piecewise quadratic.
# ----------------------------------------------------------------------------
def _argmin_piecewise_quadratic(g1, g2, lam_w, c):
    """argmin_mu g1 mu + 1/2 g2 mu^2 + lam_w |c + mu| by candidate enumeration."""
    phi = lambda mu: g1 * mu + 0.5 * g2 * mu * mu + lam_w * abs(c + mu)
    cands = [-c, -(g1 + lam_w) / g2, -(g1 - lam_w) / g2]
    return min(cands, key=phi)


@pytest.mark.parametrize("ij", [(1, 1), (0, 2), (2, 3)])
def test_lambda_cd_step_is_1d_argmin(oracle_lib, ij):
    o = oracle_lib
    rng = np.random.default_rng(10 + ij[0] * 7 + ij[1])
    p, q = 3, 4
    X, Y = random_problem(p, q, 20, seed=11)
    S = o.stats(X, Y)
    Lam, Theta = random_state(p, q, rng)
    GL, _, Sig, Psi = o.gradient(S, Lam, Theta)
    lam = 0.05
    i, j = ij
    act = np.zeros((q, q), bool)
    act[i, j] = True
    D = o.lambda_direction(Sig, Psi, GL, Lam, act, lam)
    E = np.zeros((q, q))
    E[i, j] = E[j, i] = 1.0
    eps = 1e-4
    g0 = _g(o, S, Lam, Theta)
    gp, gm = _g(o, S, Lam + eps * E, Theta), _g(o, S, Lam - eps * E, Theta)
    g1, g2 = (gp - gm) / (2 * eps), (gp - 2 * g0 + gm) / eps**2
    w = 1.0 if i == j else 2.0                       # both triangles are penalized
    mu = _argmin_piecewise_quadratic(g1, g2, lam * w, Lam[i, j])
    assert D[i, j] == pytest.approx(mu, rel=1e-5, abs=1e-8)
    assert D[j, i] == D[i, j]
    assert np.count_nonzero(D) == (1 if i == j else 2) or mu == 0


def test_lambda_cd_second_coordinate_sees_first(oracle_lib):
    """After a first coordinate moves, the second step minimises the model at
    the updated D -- pins the maintained U = D Sigma (b correction terms)."""
    o = oracle_lib
    rng = np.random.default_rng(20)
    p, q = 3, 4
    X, Y = random_problem(p, q, 20, seed=21)
    S = o.stats(X, Y)
    Lam, Theta = random_state(p, q, rng)
    GL, _, Sig, Psi = o.gradient(S, Lam, Theta)
    lam = 0.01
    (i1, j1), (i2, j2) = (0, 1), (1, 3)            # lexicographic order: first (0,1), then (1,3)
    act = np.zeros((q, q), bool)
    act[i1, j1] = act[i2, j2] = True
    D = o.lambda_direction(Sig, Psi, GL, Lam, act, lam)
    D1 = np.zeros((q, q))
    D1[i1, j1] = D1[j1, i1] = D[i1, j1]
    E = np.zeros((q, q))
    E[i2, j2] = E[j2, i2] = 1.0
    eps = 1e-3
    gf = lambda A: _g(o, S, Lam + A, Theta)
    # model m(mu) = g'(D1 + mu E) + 1/2 g''(D1 + mu E): linear coefficient
    # g'[E] + g''[D1, E], quadratic coefficient g''[E, E] (all by central differences)
    g1E = (gf(eps * E) - gf(-eps * E)) / (2 * eps)
    gEE = (gf(eps * E) - 2 * gf(0 * E) + gf(-eps * E)) / eps**2
    gDE = (gf(eps * (D1 + E)) - gf(eps * (D1 - E)) - gf(eps * (-D1 + E)) + gf(-eps * (D1 + E))) \
        / (4 * eps**2)
    mu = _argmin_piecewise_quadratic(g1E + gDE, gEE, 2 * lam, Lam[i2, j2])
    assert D[i2, j2] == pytest.approx(mu, rel=1e-4, abs=1e-7)


def test_lambda_cd_passes_solve_newton_subproblem(oracle_lib):
    """Repeated passes converge to the minimiser of the l1-penalised quadratic
    model of Eq. (6) over the active set.  Its optimality conditions are checked
    with the model gradient b = G + H[D] built from central differences of the
    gradient map (H[D] = d/de G(Lambda + e D)), not from the CD's own update
    formulas: for active (i, j), b_ij = -lam sign(Lambda + D)_ij where
    Lambda + D is nonzero and |b_ij| <= lam where it is zero."""
    o = oracle_lib
    rng = np.random.default_rng(25)
    p, q = 4, 5
    X, Y = random_problem(p, q, 30, seed=26)
    S = o.stats(X, Y)
    Lam, Theta = random_state(p, q, rng)
    GL, _, Sig, Psi = o.gradient(S, Lam, Theta)
    lam = 0.05
    act = np.ones((q, q), bool)
    act[0, 3] = act[3, 0] = False                   # one inactive pair stays at zero
    D = o.lambda_direction(Sig, Psi, GL, Lam, act, lam, passes=4000)
    assert D[0, 3] == 0.0 and D[3, 0] == 0.0
    eps = 1e-6                                      # truncation error ~3e-9 here
    Gp = o.gradient(S, Lam + eps * D, Theta)[0]
    Gm = o.gradient(S, Lam - eps * D, Theta)[0]
    b = GL + (Gp - Gm) / (2 * eps)
    x = Lam + D
    nz = act & (np.abs(x) > 1e-12)
    zero = act & ~nz
    assert nz.sum() > 0
    np.testing.assert_allclose(b[nz], -lam * np.sign(x[nz]), rtol=0, atol=1e-7)
    assert np.all(np.abs(b[zero]) <= lam + 1e-7)
    # one pass is not yet at the solution on this instance (the pin is not vacuous)
    D1 = o.lambda_direction(Sig, Psi, GL, Lam, act, lam, passes=1)
    assert np.abs(D1 - D).max() > 1e-6


def test_theta_cd_steps_are_exact_minimisers(oracle_lib):
    """g is quadratic in Theta; sequential steps on two coordinates of the same
    row and one of another row must each minimise f exactly along its axis."""
    o = oracle_lib
    rng = np.random.default_rng(30)
    p, q = 4, 3
    X, Y = random_problem(p, q, 20, seed=31)
    S = o.stats(X, Y)
    Lam, Theta0 = random_state(p, q, rng)
    Sig = np.linalg.inv(Lam)
    lam = 0.05
    coords = [(0, 1), (0, 2), (2, 0)]
    act = np.zeros((p, q), bool)
    cur = Theta0.copy()
    for (i, j) in coords:
        act[:] = False
        act[i, j] = True
        new = o.theta_sweep(S, Sig, act, lam, cur)
        E = np.zeros((p, q))
        E[i, j] = 1.0
        h = 1e-2
        fp = o.objective(S, Lam, cur + h * E, 0, 0)
        f0 = o.objective(S, Lam, cur, 0, 0)
        fm = o.objective(S, Lam, cur - h * E, 0, 0)
        g1, g2 = (fp - fm) / (2 * h), (fp - 2 * f0 + fm) / h**2      # exact for a quadratic
        mu = _argmin_piecewise_quadratic(g1, g2, lam, cur[i, j])
        assert new[i, j] - cur[i, j] == pytest.approx(mu, rel=1e-7, abs=1e-10)
        cur = new
    # and the whole pass in one call reproduces the same sequence
    act[:] = False
    for (i, j) in coords:
        act[i, j] = True
    np.testing.assert_allclose(o.theta_sweep(S, Sig, act, lam, Theta0), cur, rtol=1e-12,
                               atol=1e-14)


# ----------------------------------------------------------------------------
# Closed forms and reductions to textbook problems.
# ----------------------------------------------------------------------------
def test_closed_form_unpenalised(oracle_lib):
    """lambda = 0, n > p + q: B = Sxx^{-1} Sxy = -Theta Sigma (OLS), Sigma* is the
    residual covariance Syy - Sxy^T Sxx^{-1} Sxy, and f* = q + log det Sigma*."""
    o = oracle_lib
    p, q, n = 4, 3, 60
    X, Y = random_problem(p, q, n, seed=40)
    r = o.solve(X, Y, 0.0, 0.0, tol=1e-13, max_iter=3000, stall_iters=5)
    Sxx, Sxy, Syy = X.T @ X / n, X.T @ Y / n, Y.T @ Y / n
    B = np.linalg.solve(Sxx, Sxy)
    Sig_star = Syy - Sxy.T @ B
    np.testing.assert_allclose(np.linalg.inv(r.Lambda), Sig_star, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(-r.Theta @ np.linalg.inv(r.Lambda), B, rtol=1e-8, atol=1e-10)
    assert r.f == pytest.approx(q + np.linalg.slogdet(Sig_star)[1], rel=1e-12)


def test_theta_zero_regime_diagonal_closed_form(oracle_lib):
    """lamT >= 2 max|Sxy| forces Theta* = 0; with lamL >= max_{i!=j}|Syy_ij| as
    well, Lambda* = diag(1 / (Syy_ii + lamL))."""
    o = oracle_lib
    X, Y = random_problem(5, 4, 40, seed=41)
    Sxx, Sxy, Syy = o.stats(X, Y)
    lamT = 2 * np.abs(Sxy).max() * 1.01
    off = np.abs(Syy - np.diag(np.diag(Syy))).max()
    lamL = off * 1.01
    r = o.solve(X, Y, lamL, lamT, tol=1e-13, max_iter=500, stall_iters=5)
    assert np.all(r.Theta == 0)
    np.testing.assert_allclose(r.Lambda, np.diag(1.0 / (np.diag(Syy) + lamL)), rtol=1e-10,
                               atol=1e-12)


def test_theta_zero_regime_is_graphical_lasso(oracle_lib):
    """With Theta* = 0 the Lambda problem is the graphical lasso with a penalised
    diagonal, i.e. sklearn's graphical_lasso (unpenalised diagonal) on Syy + lamL I."""
    from sklearn.covariance import graphical_lasso
    o = oracle_lib
    X, Y = random_problem(4, 6, 50, seed=42, noise=1.0)
    Sxx, Sxy, Syy = o.stats(X, Y)
    lamT = 2 * np.abs(Sxy).max() * 1.01
    lamL = 0.25 * np.abs(Syy - np.diag(np.diag(Syy))).max()
    r = o.solve(X, Y, lamL, lamT, tol=1e-14, max_iter=3000, stall_iters=5)
    assert np.all(r.Theta == 0)
    _, prec = graphical_lasso(Syy + lamL * np.eye(6), alpha=lamL, tol=1e-12, max_iter=10000,
                              enet_tol=1e-12)
    np.testing.assert_allclose(r.Lambda, prec, rtol=1e-6, atol=1e-7)
    assert np.count_nonzero(np.abs(r.Lambda) > 1e-8) == np.count_nonzero(np.abs(prec) > 1e-8)


def _lasso_brute_force(X, y, lamT):
    """Exact minimiser of (1/n)||y - X b||^2 + lamT ||b||_1 by enumerating sign patterns."""
    n, p = X.shape
    best, best_b = np.inf, None
    for signs in itertools.product((-1, 0, 1), repeat=p):
        s = np.array(signs, float)
        S = np.flatnonzero(s)
        b = np.zeros(p)
        if S.size:
            A = X[:, S].T @ X[:, S] / n
            rhs = X[:, S].T @ y / n - 0.5 * lamT * s[S]
            bS = np.linalg.solve(A, rhs)
            if np.any(np.sign(bS) != s[S]):
                continue
            b[S] = bS
        K = np.sum((y - X @ b) ** 2) / n + lamT * np.abs(b).sum()
        if K < best:
            best, best_b = K, b
    return best_b, best


def test_single_output_reduces_to_lasso(oracle_lib):
    """q = 1: with b = -theta / Lambda_11, f = -log L + L K(b) with
    K(b) = (1/n)||y - Xb||^2 + lamT ||b||_1 + lamL; so b* is the lasso
    solution, Lambda* = 1 / K(b*), Theta* = -Lambda* b*, f* = 1 + log K(b*)."""
    from sklearn.linear_model import Lasso
    o = oracle_lib
    n, p = 40, 6
    X, Y = random_problem(p, 1, n, seed=43, theta_density=0.5)
    lamL, lamT = 0.03, 0.15
    r = o.solve(X, Y, lamL, lamT, tol=1e-14, max_iter=5000, stall_iters=5)
    b_bf, Kmin = _lasso_brute_force(X, Y[:, 0], lamT)
    K = Kmin + lamL
    assert r.Lambda[0, 0] == pytest.approx(1.0 / K, rel=1e-9)
    np.testing.assert_allclose(r.Theta[:, 0], -b_bf / K, rtol=1e-8, atol=1e-10)
    assert r.f == pytest.approx(1.0 + np.log(K), rel=1e-12)
    las = Lasso(alpha=lamT / 2, fit_intercept=False, tol=1e-14, max_iter=200000).fit(X, Y[:, 0])
    np.testing.assert_allclose(las.coef_, b_bf, rtol=1e-6, atol=1e-8)


def test_diagonal_lambda_regime_is_independent_lassos(oracle_lib):
    """When lamL >= max_{i!=j} |Syy_ij - b_i^T Sxx b_j| (checked after the fact)
    the solution is q independent lassos with diagonal Lambda."""
    from sklearn.linear_model import Lasso
    o = oracle_lib
    rng = np.random.default_rng(44)
    n, p, q = 200, 5, 3
    X = rng.standard_normal((n, p))
    B = synth.dense_theta(p, q, 0.5, rng)
    Y = X @ B + 0.5 * rng.standard_normal((n, q))
    lamL, lamT = 0.5, 0.05
    r = o.solve(X, Y, lamL, lamT, tol=1e-14, max_iter=5000, stall_iters=5)
    Sxx = X.T @ X / n
    bs, Ks = [], []
    for j in range(q):
        b = Lasso(alpha=lamT / 2, fit_intercept=False, tol=1e-15, max_iter=500000).fit(
            X, Y[:, j]).coef_
        bs.append(b)
        Ks.append(np.sum((Y[:, j] - X @ b) ** 2) / n + lamT * np.abs(b).sum() + lamL)
    bmat = np.array(bs).T
    Syy = Y.T @ Y / n
    G = Syy - bmat.T @ Sxx @ bmat
    assert np.abs(G - np.diag(np.diag(G))).max() < lamL      # regime holds
    np.testing.assert_allclose(r.Lambda, np.diag(1.0 / np.array(Ks)), rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose(r.Theta, -bmat / np.array(Ks), rtol=1e-5, atol=1e-8)


# ----------------------------------------------------------------------------
# Independent solver: nonmonotone proximal gradient with Barzilai-Borwein steps
# (SpaRSA, Wright-Nowak-Figueiredo 2009) that keeps Lambda positive definite,
# run to a tiny step on problems with p, q <= 6.  It shares nothing with the
# oracle but the objective's definition.
# ----------------------------------------------------------------------------
def _prox_grad(X, Y, lamL, lamT, iters=20000, tol=1e-13):
    n = X.shape[0]
    Sxx, Sxy, Syy = X.T @ X / n, X.T @ Y / n, Y.T @ Y / n
    q, p = Y.shape[1], X.shape[1]

    def smooth(L, T):
        try:
            C = np.linalg.cholesky(L)
        except np.linalg.LinAlgError:
            return np.inf, None, None
        Ci = np.linalg.inv(C)
        Sig = Ci.T @ Ci
        Gam = Sxx @ T @ Sig
        val = -2 * np.log(np.diag(C)).sum() + np.sum(Syy * L) + 2 * np.sum(Sxy * T) \
            + np.sum(Sig * (T.T @ Sxx @ T))
        GL = Syy - Sig - Sig @ T.T @ Gam
        return val, (GL + GL.T) / 2, 2 * Sxy + 2 * Gam

    pen = lambda L, T: lamL * np.abs(L).sum() + lamT * np.abs(T).sum()
    st = lambda w, r: np.sign(w) * np.maximum(np.abs(w) - r, 0)
    L, T = np.eye(q), np.zeros((p, q))
    g, GL, GT = smooth(L, T)
    hist = [g + pen(L, T)]
    step = 1.0
    for _ in range(iters):
        while True:                                   # backtrack: PD + nonmonotone decrease
            nL, nT = st(L - step * GL, step * lamL), st(T - step * GT, step * lamT)
            ng, nGL, nGT = smooth(nL, nT)
            dL, dT = nL - L, nT - T
            dd = np.sum(dL * dL) + np.sum(dT * dT)
            if ng < np.inf and ng + pen(nL, nT) <= max(hist[-10:]) - 1e-4 / (2 * step) * dd:
                break
            step *= 0.5
        sy = np.sum(dL * (nGL - GL)) + np.sum(dT * (nGT - GT))
        L, T, GL, GT = nL, nT, nGL, nGT
        hist.append(ng + pen(L, T))
        step = min(max(dd / sy if sy > 0 else 1.0, 1e-10), 1e10)   # BB step
        if dd < tol * tol:
            break
    return L, T, hist[-1]


# The last three draws have fewer samples than inputs and outputs together
# (n < p + q; two of them n < p), the regime of
# the larger benchmark workloads: there the objective is nearly flat along
# some directions, the oracle's coordinate descent takes thousands of
# iterations, and the proximal-gradient solver stops at a KKT residual near
# 1e-8 with parameters ~1e-7 from the optimum while its objective agrees to
# 1e-13.  The oracle is held to the tighter KKT bound itself.
@pytest.mark.parametrize("seed,p,q,n", [(50, 3, 4, 30), (51, 5, 3, 30), (52, 6, 6, 30),
                                        (53, 9, 4, 7), (54, 8, 6, 10), (55, 12, 3, 9)])
def test_agrees_with_proximal_gradient(oracle_lib, seed, p, q, n):
    X, Y = random_problem(p, q, n, seed=seed)
    lamL, lamT = 0.06, 0.09
    flat = n < p + q
    r = oracle_lib.solve(X, Y, lamL, lamT, tol=1e-14, max_iter=200000, stall_iters=5)
    assert r.status in (oracle_lib.ORC_OK, oracle_lib.ORC_STALLED)
    GL, GT = _numpy_gradient(X, Y, r.Lambda, r.Theta)
    assert max(_kkt_violation(GL, r.Lambda, lamL), _kkt_violation(GT, r.Theta, lamT)) < 1e-9
    L, T, f = _prox_grad(X, Y, lamL, lamT, iters=200000, tol=1e-15 if flat else 1e-13)
    GL, GT = _numpy_gradient(X, Y, L, T)
    assert max(_kkt_violation(GL, L, lamL), _kkt_violation(GT, T, lamT)) < (
        1e-7 if flat else 1e-9)
    assert r.f == pytest.approx(f, rel=1e-12)
    atol = 1e-5 if flat else 1e-8
    np.testing.assert_allclose(r.Lambda, L, atol=atol)
    np.testing.assert_allclose(r.Theta, T, atol=atol)
    for a, b in ((r.Lambda, L), (r.Theta, T)):     # supports outside [1e-7, 1e-5]
        clear = (np.abs(a) < 1e-7) | (np.abs(a) > 1e-5)
        assert np.array_equal((np.abs(a) > 1e-6)[clear], (np.abs(b) > 1e-6)[clear])


# ----------------------------------------------------------------------------
# Optimality and invariants on the benchmark generator's smallest workload.
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def chain40_solution(oracle_lib):
    pr = synth.workload("chain40")
    r = oracle_lib.solve(pr.X, pr.Y, pr.lam_Lambda, pr.lam_Theta, tol=1e-14, max_iter=2000,
                         stall_iters=3)
    return pr, r


def _numpy_gradient(X, Y, Lam, Theta):
    n = X.shape[0]
    Sxx, Sxy, Syy = X.T @ X / n, X.T @ Y / n, Y.T @ Y / n
    Sig = np.linalg.inv(Lam)
    Gam = Sxx @ Theta @ Sig
    return Syy - Sig - Sig @ Theta.T @ Gam, 2 * Sxy + 2 * Gam


def _kkt_violation(G, P, lam):
    nz = P != 0
    v_nz = np.abs(G[nz] + lam * np.sign(P[nz]))
    v_z = np.maximum(np.abs(G[~nz]) - lam, 0)
    return max(v_nz.max(initial=0), v_z.max(initial=0))


def test_kkt_at_solution(chain40_solution):
    pr, r = chain40_solution
    GL, GT = _numpy_gradient(pr.X, pr.Y, r.Lambda, r.Theta)
    assert _kkt_violation(GL, r.Lambda, pr.lam_Lambda) < 1e-8
    assert _kkt_violation(GT, r.Theta, pr.lam_Theta) < 1e-8
    # diagonal: Sigma_ii + Psi_ii = Syy_ii + lamL (Lambda_ii > 0)
    assert np.all(np.diag(r.Lambda) > 0)


def test_monotone_pd_symmetric(chain40_solution):
    pr, r = chain40_solution
    f = r.trace["f"]
    assert np.all(np.diff(f) <= 1e-12 * np.abs(f[1:]))
    assert np.allclose(r.Lambda, r.Lambda.T, rtol=0, atol=0)
    assert np.linalg.eigvalsh(r.Lambda).min() > 0
    assert r.status in (0, 2)


def test_permutation_equivariance(oracle_lib, chain40_solution):
    pr, r = chain40_solution
    rng = np.random.default_rng(60)
    px, py = rng.permutation(pr.p), rng.permutation(pr.q)
    r2 = oracle_lib.solve(pr.X[:, px], pr.Y[:, py], pr.lam_Lambda, pr.lam_Theta, tol=1e-14,
                          max_iter=2000, stall_iters=3)
    assert r2.f == pytest.approx(r.f, rel=1e-11)
    np.testing.assert_allclose(r2.Lambda, r.Lambda[np.ix_(py, py)], atol=1e-7)
    np.testing.assert_allclose(r2.Theta, r.Theta[np.ix_(px, py)], atol=1e-7)


def test_x_scaling_map(oracle_lib):
    """Theta(cX, lamT) = Theta(X, lamT / c) / c and Lambda unchanged."""
    X, Y = random_problem(5, 4, 40, seed=61)
    c, lamL, lamT = 2.5, 0.05, 0.08
    a = oracle_lib.solve(c * X, Y, lamL, lamT, tol=1e-14, max_iter=3000, stall_iters=5)
    b = oracle_lib.solve(X, Y, lamL, lamT / c, tol=1e-14, max_iter=3000, stall_iters=5)
    assert a.f == pytest.approx(b.f, rel=1e-11)
    np.testing.assert_allclose(a.Lambda, b.Lambda, atol=1e-8)
    np.testing.assert_allclose(a.Theta, b.Theta / c, atol=1e-8)


def test_warm_start_from_other_point_same_optimum(oracle_lib, chain40_solution):
    pr, r = chain40_solution
    rng = np.random.default_rng(62)
    L0 = synth.random_spd(pr.q, rng)
    T0 = synth.dense_theta(pr.p, pr.q, 0.2, rng)
    r2 = oracle_lib.solve(pr.X, pr.Y, pr.lam_Lambda, pr.lam_Theta, tol=1e-14, max_iter=3000,
                          stall_iters=3, Lambda0=L0, Theta0=T0)
    assert r2.f == pytest.approx(r.f, rel=1e-11)
    np.testing.assert_allclose(r2.Lambda, r.Lambda, atol=1e-7)
