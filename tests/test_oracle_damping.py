"""Pins of the damped selection (select="newton_first", the reading this library
gives Sec. 5's "more refined step damping"): the Newton candidate alone is
costed and kept iff it does not raise the column's (row's) eq. (5) objective,
else the MU candidate is kept uncosted.  CPU only."""
import numpy as np
import pytest

import oracle
from oracle import dna_oracle as O
from paper_1301_3389_amd import synth


def _col_objective(V, W, H, lam=0.0):
    """Eq. (5) per column, from its definition: sum v log(v/z) - v + z over the
    column, plus lambda sum_r h_r."""
    V, Z = np.asarray(V, float), np.asarray(W, float) @ np.asarray(H, float)
    pos = V > 0
    t = np.where(pos, V * np.log(np.where(pos, V, 1.0) / np.where(pos, Z, 1.0)), 0.0) - V + Z
    return t.sum(axis=0) + lam * np.asarray(H, float).sum(axis=0)


def _row_objective(V, W, H, rho=0.0):
    return _col_objective(np.asarray(V).T, np.asarray(H).T, np.asarray(W).T, rho)


@pytest.mark.parametrize("lam", [0.0, 0.3])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_newton_first_never_raises_the_column_objective(seed, lam):
    """Every column's eq. (5) objective after the damped H step is at or below
    the current one (MU is monotone, Newton is kept only when it is), and the
    kept column is exactly one of the two candidates."""
    w = synth.random_problem(80, 120, 7, seed, zero_frac=0.1)
    V, W, H = w.V.astype(float), w.W.astype(float), w.H.astype(float)
    r = oracle.h_step(V, W, H, lam=lam, select="newton_first")
    before = _col_objective(V, W, H, lam)
    after = _col_objective(V, W, r.X, lam)
    assert np.all(after <= before + 1e-9 * np.abs(before))
    kept = np.where(r.chose_newton[None, :], r.X_newton, r.X_mu)
    np.testing.assert_array_equal(r.X, kept)
    # the margin is the objective difference, from the definition
    np.testing.assert_allclose(r.margin, before - _col_objective(V, W, r.X_newton, lam), rtol=1e-9,
                               atol=1e-9 * np.abs(before).max())
    assert np.all(np.isnan(r.d_mu)) and np.all(np.isnan(r.d_sel[~r.chose_newton]))


@pytest.mark.parametrize("seed", [4, 5])
def test_newton_first_w_step_never_raises_the_row_objective(seed):
    w = synth.random_problem(90, 70, 6, seed, zero_frac=0.1)
    V, W, H = w.V.astype(float), w.W.astype(float), w.H.astype(float)
    r = oracle.w_step(V, W, H, rho=0.2, select="newton_first")
    before = _row_objective(V, W, H, 0.2)
    after = _row_objective(V, r.X, H, 0.2)
    assert np.all(after <= before + 1e-9 * np.abs(before))
    # W step = H step on the transposed problem (Sec. 2)
    rt = oracle.h_step(V.T, H.T, W.T, lam=0.2, select="newton_first")
    np.testing.assert_array_equal(r.chose_newton, rt.chose_newton)
    np.testing.assert_allclose(r.X, rt.X.T, rtol=1e-12)


@pytest.mark.parametrize("seed", [6, 7, 8])
def test_newton_first_keeps_newton_wherever_the_paper_rule_does(seed):
    """Where Algorithm 1's rule keeps Newton (d_DNA < d_MU), Newton is also
    below the current objective (MU never raises it), so the damped rule keeps
    the same Newton column: its Newton set contains the paper's, with equal
    values there; elsewhere it may keep Newton where MU was lower."""
    w = synth.random_problem(100, 150, 9, seed, zero_frac=0.05)
    V, W, H = w.V.astype(float), w.W.astype(float), w.H.astype(float)
    full = oracle.h_step(V, W, H)
    damp = oracle.h_step(V, W, H, select="newton_first")
    assert np.all(damp.chose_newton[full.chose_newton])
    np.testing.assert_array_equal(damp.X[:, full.chose_newton], full.X[:, full.chose_newton])
    np.testing.assert_array_equal(damp.X_newton, full.X_newton)
    np.testing.assert_array_equal(damp.X_mu, full.X_mu)


def test_newton_first_falls_back_on_a_real_trajectory():
    """40 damped iterations on the 1024 x 512 slab of the N=1024 T=8192 R=64
    workload: late in the run some Newton columns would raise the cost (the
    diagonal Hessian ignores the coupling between ranks); there the damped
    rule keeps the MU candidate, whose objective never rises, and the margin
    (current minus Newton objective) is negative.  Every column's eq. (5)
    objective is non-increasing at every H step."""
    w = synth.config2()
    V = w.V[:, :512].astype(float)
    W, H = oracle.normalize(w.W.astype(float), w.H[:, :512].astype(float), 0)
    fallbacks = 0
    for _ in range(40):
        before = _col_objective(V, W, H)
        r = oracle.h_step(V, W, H, select="newton_first")
        after = _col_objective(V, W, r.X)
        assert np.all(after <= before + 1e-9 * np.abs(before))
        fb = ~r.chose_newton
        fallbacks += int(fb.sum())
        assert np.all(r.margin[fb] < 0)
        np.testing.assert_array_equal(r.X[:, fb], r.X_mu[:, fb])
        W, H = oracle.normalize(W, r.X, 1)
        W = oracle.w_step(V, W, H, select="newton_first").X
        W, H = oracle.normalize(W, H, 0)
    assert fallbacks > 0


def test_newton_first_r1_takes_the_exact_minimiser():
    """R = 1: the renormalised Newton candidate is the exact minimiser S/c of the
    column objective, never above the current one: always kept."""
    rng = np.random.default_rng(9)
    W = rng.uniform(0.1, 1.0, (30, 1))
    V = rng.poisson(5.0, (30, 40)).astype(float) + 0.5
    H = rng.uniform(0.1, 3.0, (1, 40))
    r = oracle.h_step(V, W, H, select="newton_first")
    assert np.all(r.chose_newton)
    np.testing.assert_allclose(r.X[0], V.sum(0) / W.sum(), rtol=1e-12)


@pytest.mark.parametrize("rho,lam", [(0.0, 0.0), (0.1, 0.1)])
def test_newton_first_trajectory_is_monotone(rho, lam):
    """Whole iterations with the damped selection on workload 1: eq. (2) never
    rises (checked after every iteration), and the KL reached after 20
    iterations lies between MU's and the paper's DNA's at most a few percent
    above DNA's (measured, not a bound of the method)."""
    w = synth.config1()
    d = oracle.fit_dna(w.V, w.W, w.H, 20, rho=rho, lam=lam, select="newton_first")
    obj = np.array(d.obj)
    assert np.all(np.diff(obj) <= 1e-9 * np.abs(obj[:-1]))
    if rho == 0.0:
        full = oracle.fit_dna(w.V, w.W, w.H, 20)
        mu = oracle.fit_mu(w.V, w.W, w.H, 20)
        assert d.kl[-1] < mu.kl[-1]
        assert d.kl[-1] <= 1.05 * full.kl[-1]
