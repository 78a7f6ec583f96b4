"""Pins of the regularised oracle (eq. 2-5 with rho, lambda > 0: eq. 7, 9, 10,
11, 14 with c_r + lambda, and the normalisation reading).

Each check compares the oracle with something it does not compute itself: the
objective of eq. (2) / eq. (5) evaluated from its definition, its derivatives by
central differences, a closed-form minimiser, a generic bound-constrained
solver, or a brute-force scan.
"""
import numpy as np
import pytest

import oracle
from paper_1301_3389_amd import synth


def _col_obj(v, W, h, lam):
    """Eq. (5) for one column: d_KL(v, W h) + lambda 1^t h, from its definition
    (terms with v = 0 contribute z only)."""
    z = W @ h
    pos = v > 0
    return float(np.sum(v[pos] * np.log(v[pos] / z[pos])) - v.sum() + z.sum() + lam * h.sum())


def _full_obj(V, W, H, rho, lam):
    """Eq. (2) from its definition."""
    Z = W @ H
    pos = V > 0
    return float(np.sum(V[pos] * np.log(V[pos] / Z[pos])) - V.sum() + Z.sum() + rho * W.sum() + lam * H.sum())


def _problem(N, T, R, seed, zero_frac=0.2):
    w = synth.random_problem(N, T, R, seed, zero_frac=zero_frac)
    return [x.astype(float) for x in (w.V, w.W, w.H)]


@pytest.mark.parametrize("lam", [0.0, 0.5, 3.0])
def test_r1_regularised_minimiser(lam):
    """R = 1: eq. (5) is sum v log(v/(w h)) - sum v + (c + lambda) h, so its
    minimiser is h* = sum v / (c + lambda).  One H half-step lands on it from
    any h > 0: MU gives h (1 + a) = sum v / (c + lambda) and eq. (10) maps any
    positive Newton candidate onto the same point.  The W step mirrors it with
    w*_n = sum_t v_nt / (g + rho)."""
    rng = np.random.default_rng(1)
    N, T = 9, 5
    W = rng.uniform(0.1, 2.0, (N, 1))
    V = rng.uniform(0.0, 3.0, (N, T))
    V[V < 0.5] = 0.0
    V[:, 0] = np.maximum(V[:, 0], 1.0)
    H = rng.uniform(0.1, 5.0, (1, T))
    hstar = V.sum(0) / (W.sum() + lam)
    r = oracle.h_step(V, W, H, lam=lam)
    for X in (r.X, r.X_mu, r.X_newton):
        np.testing.assert_allclose(X[0], hstar, rtol=1e-12)
    for t in range(T):
        if hstar[t] == 0:
            continue
        grid = hstar[t] * np.linspace(0.5, 1.5, 2001)
        best = min(_col_obj(V[:, t], W, np.array([g]), lam) for g in grid)
        assert _col_obj(V[:, t], W, r.X[:, t], lam) <= best + 1e-12 * abs(best)
    q = oracle.w_step(V, W, H, rho=lam)
    np.testing.assert_allclose(q.X[:, 0], V.sum(1) / (H.sum() + lam), rtol=1e-12)


def test_eq9_and_selection_on_the_regularised_cost():
    """Both candidates satisfy eq. (9), sum_r (c_r + lambda) x_r = sum_n v_n, so
    selecting on the log-ratio sums (steps 9, 14) is selecting on eq. (5): the
    margin d_MU - d_DNA equals the eq. (5) difference of the two candidates.
    The kept column never has a larger eq. (5) value than the input column
    (MU does not increase eq. 5, Sec. 2.1)."""
    V, W, H = _problem(40, 30, 6, 3, zero_frac=0.3)
    W = W * 2.5
    lam = 0.7
    r = oracle.h_step(V, W, H, lam=lam)
    c = W.sum(0)
    for X in (r.X_mu, r.X_newton):
        np.testing.assert_allclose((c + lam) @ X, V.sum(0), rtol=1e-12)
    T = V.shape[1]
    f_mu = np.array([_col_obj(V[:, t], W, r.X_mu[:, t], lam) for t in range(T)])
    f_nr = np.array([_col_obj(V[:, t], W, r.X_newton[:, t], lam) for t in range(T)])
    f_in = np.array([_col_obj(V[:, t], W, H[:, t], lam) for t in range(T)])
    f_sel = np.array([_col_obj(V[:, t], W, r.X[:, t], lam) for t in range(T)])
    scale = np.abs(f_in) + V.sum(0)
    np.testing.assert_allclose(r.margin, f_mu - f_nr, rtol=0, atol=1e-10 * scale.max())
    clear = np.abs(f_mu - f_nr) > 1e-9 * scale
    assert np.array_equal(r.chose_newton[clear], (f_nr < f_mu)[clear])
    assert np.all(f_sel <= f_in + 1e-12 * scale)
    assert np.all(f_mu <= f_in + 1e-12 * scale)


def test_regularised_gradient_and_hessian_by_finite_differences():
    """-(c_r + lambda) a_r is the partial derivative of eq. (5) in h_r (the KKT
    expression of Sec. 2, eq. 6-7) and (c_r + lambda) b_r its second partial
    derivative (eq. 13-14): central differences of eq. (5)."""
    V, W, H = _problem(20, 6, 4, 5, zero_frac=0.1)
    W = W * 1.7
    H = H + 0.2
    lam = 1.3
    r = oracle.h_step(V, W, H, lam=lam)
    ck = W.sum(0) + lam
    for t in range(H.shape[1]):
        v = V[:, t]
        for k in range(H.shape[0]):
            h = H[:, t].copy()
            d = 1e-4 * h[k]
            hp, hm = h.copy(), h.copy()
            hp[k] += d
            hm[k] -= d
            fp, f0, fm = _col_obj(v, W, hp, lam), _col_obj(v, W, h, lam), _col_obj(v, W, hm, lam)
            d1 = (fp - fm) / (2 * d)
            d2 = (fp - 2 * f0 + fm) / (d * d)
            assert d1 == pytest.approx(-ck[k] * r.A[k, t], rel=1e-6, abs=1e-8)
            assert d2 == pytest.approx(ck[k] * r.B[k, t], rel=1e-4)


@pytest.mark.parametrize("lam", [0.3, 4.0])
def test_regularised_subproblem_matches_external_solver(lam):
    """Eq. (5) with lambda > 0 is convex in h: H-only DNA runs and long MU runs
    reach the minimiser a generic bound-constrained solver finds, and the KKT
    conditions (eq. 8) hold there.  lambda = 4 drives some h_r to 0."""
    scipy_opt = pytest.importorskip("scipy.optimize")
    rng = np.random.default_rng(11)
    N, R, T = 8, 3, 4
    W = rng.uniform(0.1, 1.0, (N, R))
    Htrue = rng.uniform(0.5, 2.0, (R, T))
    V = (W @ Htrue) * rng.uniform(0.9, 1.1, (N, T))
    H = np.ones((R, T))
    for _ in range(300):
        H = oracle.h_step(V, W, H, lam=lam).X
    Hm = np.ones((R, T))
    for _ in range(50000):
        Hm, _ = oracle.mu_h_step(V, W, Hm, lam=lam)
    c = W.sum(0)
    for t in range(T):
        v = V[:, t]
        res = scipy_opt.minimize(lambda h: _col_obj(v, W, h, lam), np.ones(R),
                                 jac=lambda h: c + lam - W.T @ (v / (W @ h)), method="L-BFGS-B",
                                 bounds=[(1e-300, None)] * R,
                                 options={"ftol": 1e-15, "gtol": 1e-13, "maxiter": 10000})
        np.testing.assert_allclose(H[:, t], res.x, rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(Hm[:, t], res.x, rtol=1e-5, atol=1e-6)
    r = oracle.h_step(V, W, H, lam=lam)
    assert np.max(np.abs(r.A * H)) < 1e-9
    assert np.all(r.A[H < 1e-8] <= 1e-9)
    if lam == 4.0:
        assert np.any(H < 1e-8)


def test_balanced_normalisation_minimises_the_penalty():
    """With rho, lambda > 0 the normalisation leaves W H unchanged, makes
    rho C_r = lambda G_r, and no other per-component scale gives a smaller
    rho sum w + lambda sum h (scan over 4001 scales spanning 10^-3 .. 10^3)."""
    _, W, H = _problem(30, 25, 5, 7)
    rho, lam = 0.4, 2.5
    W2, H2 = oracle.normalize(W, H, 0, rho, lam)
    W3, H3 = oracle.normalize(W, H, 1, rho, lam)
    np.testing.assert_allclose(W2, W3, rtol=1e-14)
    np.testing.assert_allclose(W2 @ H2, W @ H, rtol=1e-13)
    np.testing.assert_allclose(rho * W2.sum(0), lam * H2.sum(1), rtol=1e-13)
    C, G = W.sum(0), H.sum(1)
    grid = np.logspace(-3, 3, 4001)
    for r in range(W.shape[1]):
        best = np.min(rho * C[r] * grid + lam * G[r] / grid)
        got = rho * W2[:, r].sum() + lam * H2[r].sum()
        assert got <= best * (1 + 1e-12)
    assert rho * W2.sum() + lam * H2.sum() <= rho * W.sum() + lam * H.sum()


def test_one_sided_normalisation_fixes_the_unpenalised_scale():
    _, W, H = _problem(30, 25, 5, 8)
    for side in (0, 1):
        W2, H2 = oracle.normalize(W, H, side, rho=0.0, lam=0.8)
        np.testing.assert_allclose(W2.sum(0), 1.0, rtol=1e-14)
        np.testing.assert_allclose(W2 @ H2, W @ H, rtol=1e-13)
        W3, H3 = oracle.normalize(W, H, side, rho=0.8, lam=0.0)
        np.testing.assert_allclose(H3.sum(1), 1.0, rtol=1e-14)
        np.testing.assert_allclose(W3 @ H3, W @ H, rtol=1e-13)
    W4, H4 = oracle.normalize(W, H, 1)
    np.testing.assert_allclose(H4.sum(1), 1.0, rtol=1e-14)


@pytest.mark.parametrize("rho,lam", [(0.3, 0.6), (2.0, 0.05)])
def test_objective_non_increasing_at_every_step(rho, lam):
    """With rho, lambda > 0: eq. (2), evaluated from its definition, does not
    increase over any H half-step, normalisation or W half-step of Algorithm 1,
    and likewise under the MU-only iteration."""
    V, W, H = _problem(35, 28, 5, 9, zero_frac=0.25)
    W, H = oracle.normalize(W, H, 0, rho, lam)
    prev = _full_obj(V, W, H, rho, lam)
    for _ in range(15):
        for stage in range(4):
            if stage == 0:
                H = oracle.h_step(V, W, H, lam=lam).X
            elif stage == 1:
                W, H = oracle.normalize(W, H, 1, rho, lam)
            elif stage == 2:
                W = oracle.w_step(V, W, H, rho=rho).X
            else:
                W, H = oracle.normalize(W, H, 0, rho, lam)
            cur = _full_obj(V, W, H, rho, lam)
            assert cur <= prev + 1e-12 * abs(prev), (stage, cur, prev)
            prev = cur
    fit = oracle.fit_dna(V, W, H, 10, rho=rho, lam=lam)
    np.testing.assert_allclose(fit.obj[-1], _full_obj(V, fit.W, fit.H, rho, lam), rtol=1e-12)
    assert np.all(np.diff(fit.obj) <= 1e-12 * np.abs(fit.obj[:-1]))
    mu = oracle.fit_mu(V, W, H, 30, rho=rho, lam=lam)
    assert np.all(np.diff(mu.obj) <= 1e-12 * np.abs(mu.obj[:-1]))
    assert fit.obj[-1] < mu.obj[10]


def test_regularised_w_step_is_h_step_on_transposes():
    """Sec. 2: d(V, W H) + rho sum w = d(V^t, H^t W^t) + rho sum w, so the W step
    with rho is the H step with lambda = rho on the transposed problem."""
    V, W, H = _problem(22, 17, 4, 10)
    rho = 0.9
    a = oracle.w_step(V, W, H, rho=rho)
    b = oracle.h_step(V.T, H.T, W.T, lam=rho)
    np.testing.assert_allclose(a.X, b.X.T, rtol=1e-13)
    np.testing.assert_array_equal(a.chose_newton, b.chose_newton)
    m1, _ = oracle.mu_w_step(V, W, H, rho=rho)
    m2, _ = oracle.mu_h_step(V.T, H.T, W.T, lam=rho)
    np.testing.assert_allclose(m1, m2.T, rtol=1e-13)


def test_regularisation_shrinks_the_fixed_point():
    """At the minimiser of eq. (5), sum_r (c_r + lambda) h_r = sum v (eq. 9), so
    sum z = sum_r c_r h_r = sum v - lambda sum h: the data mass the model
    explains drops by exactly lambda sum h."""
    rng = np.random.default_rng(12)
    W = rng.uniform(0.1, 1.0, (10, 3))
    V = (W @ rng.uniform(0.5, 2.0, (3, 6))) * rng.uniform(0.9, 1.1, (10, 6))
    lam = 0.5
    H = np.ones((3, 6))
    for _ in range(200):
        H = oracle.h_step(V, W, H, lam=lam).X
    np.testing.assert_allclose((W @ H).sum(0), V.sum(0) - lam * H.sum(0), rtol=1e-10)
