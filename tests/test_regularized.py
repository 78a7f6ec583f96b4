"""Regularised DNA (eq. 2 with rho, lambda >= 0): the GPU path against the FP64
oracle run with the same weights -- half-steps, their stages, MU, the three
normalisation forms, the eq. 2 cost, whole iterations and trajectories, dense
and sparse V."""
import numpy as np
import pytest
import torch

import oracle
from paper_1301_3389_amd import synth
from parity_util import (FLOOR32, STATE_TIE, STEP_TOL, TRAJ_TOL, cost_err, gpu, host, log_result, recon_gap,
                         rel_cols, selection_report)

pytestmark = pytest.mark.gpu

SHAPES = [
    # N, T, R, zero_frac, seed
    (300, 333, 37, 0.2, 1),
    (257, 130, 10, 0.0, 2),
    (1000, 515, 64, 0.1, 4),
    (150, 170, 100, 0.1, 10),
    (200, 300, 129, 0.05, 9),
    (5, 7, 3, 0.0, 6),
]

# (rho, lambda) as fractions of the mean H row sum / mean W column sum, so that
# each weight moves the step by a visible amount whatever the problem's scale:
# lambda alone, rho alone, both.
FRACS = [(0.0, 0.4), (0.6, 0.0), (0.25, 1.5)]


def _problem(N, T, R, zf, seed):
    w = synth.random_problem(N, T, R, seed, zero_frac=zf)
    V = w.V.copy()
    V[0, :] = np.maximum(V[0, :], 1.0)
    V[:, 0] = np.maximum(V[:, 0], 1.0)
    return V, w.W, w.H


def _weights(W, H, frac):
    fr, fl = frac
    rho = fr * float(np.mean(H.astype(float).sum(axis=1)))
    lam = fl * float(np.mean(W.astype(float).sum(axis=0)))
    # the library holds the weights as float32: hand the oracle the same numbers
    return float(np.float32(rho)), float(np.float32(lam))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("frac", FRACS)
def test_reg_update(dna, shape, side, frac):
    V, W, H = _problem(*shape)
    rho, lam = _weights(W, H, frac)
    Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
    if side == 0:
        m, d, g = dna.update_H(Vg, Wg, Hg, mask=True, d_sel=True, margin=True, rho=rho, lam=lam)
        got = host(Hg)
        r = oracle.h_step(V, W, H, value_floor=FLOOR32, lam=lam)
    else:
        m, d, g = dna.update_W(Vg, Wg, Hg, mask=True, d_sel=True, margin=True, rho=rho, lam=lam)
        got = host(Wg)
        r = oracle.w_step(V, W, H, value_floor=FLOOR32, rho=rho)
    ax = 0 if side == 0 else 1
    mask = host(m).astype(bool)
    Wd, Hd = W.astype(float), H.astype(float)
    zgap = recon_gap(Wd @ r.X_mu, Wd @ r.X_newton, 0) if side == 0 else recon_gap(r.X_mu @ Hd, r.X_newton @ Hd, 1)
    rep = selection_report(mask, r.chose_newton, r.margin, r.d_mu, STATE_TIE, zgap)
    same = mask == r.chose_newton
    err = rel_cols(got, r.X, ax)[same]
    sel = r.chose_newton[None, :] if side == 0 else r.chose_newton[:, None]
    err_other = rel_cols(got, np.where(sel, r.X_mu, r.X_newton), ax)[~same]
    vsum = V.astype(float).sum(axis=ax)
    err_d = cost_err(host(d)[same], r.d_sel[same], vsum[same])
    log_result("reg_update", {"shape": shape, "side": side, "rho": rho, "lam": lam, **rep,
                              "max_err": float(err.max()) if err.size else 0.0, "err_dsel": err_d})
    assert rep["n_flips_above_tie"] == 0, rep
    assert err.size == 0 or err.max() <= STEP_TOL
    assert err_other.size == 0 or err_other.max() <= STEP_TOL
    assert err_d <= 1.0


@pytest.mark.parametrize("shape", SHAPES[:4])
@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("gemm", ["fp32", "bf16"])
def test_reg_gradient_hessian(dna, shape, side, gemm):
    """A and B of eq. (7) / (14) with c + lambda (g + rho).  BF16 products carry
    a relative error of a few 2^-8 in the sums (the bound of the unregularised
    16-bit tests); the divisor is the same float32 number."""
    V, W, H = _problem(*shape)
    rho, lam = _weights(W, H, FRACS[2])
    A, B = dna.gradient_hessian(side, gpu(V), gpu(W), gpu(H), rho=rho, lam=lam, gemm=gemm)
    r = oracle.h_step(V, W, H, lam=lam) if side == 0 else oracle.w_step(V, W, H, rho=rho)
    A, B = host(A), host(B)
    errA = np.max(np.abs(A - r.A) / (np.abs(1.0 + r.A) + 1e-30))
    errB = rel_cols(B, r.B, axis=0 if side == 0 else 1).max()
    tol = STEP_TOL if gemm == "fp32" else 4 * 2.0 ** -8
    log_result("reg_gradient_hessian", {"shape": shape, "side": side, "gemm": gemm, "errA": float(errA),
                                        "errB": float(errB)})
    assert errA <= tol and errB <= tol


@pytest.mark.parametrize("shape", SHAPES[:4])
@pytest.mark.parametrize("side", [0, 1])
def test_reg_mu_update(dna, shape, side):
    V, W, H = _problem(*shape)
    rho, lam = _weights(W, H, FRACS[2])
    Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
    dna.mu_update(side, Vg, Wg, Hg, rho=rho, lam=lam)
    if side == 0:
        ref, _ = oracle.mu_h_step(V, W, H, value_floor=FLOOR32, lam=lam)
        err = rel_cols(host(Hg), ref, 0).max()
    else:
        ref, _ = oracle.mu_w_step(V, W, H, value_floor=FLOOR32, rho=rho)
        err = rel_cols(host(Wg), ref, 1).max()
    assert err <= STEP_TOL


@pytest.mark.parametrize("shape", SHAPES[:4])
@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("frac", FRACS)
def test_reg_normalize(dna, shape, side, frac):
    """The three normalisation forms against the oracle's: W H unchanged, and
    with both weights positive rho C_r = lambda G_r afterwards."""
    V, W, H = _problem(*shape)
    rho, lam = _weights(W, H, frac)
    Wg, Hg = gpu(W), gpu(H)
    dna.normalize(side, Wg, Hg, rho=rho, lam=lam)
    Wr, Hr = oracle.normalize(W, H, side, rho, lam)
    np.testing.assert_allclose(host(Wg), Wr, rtol=3e-7)
    np.testing.assert_allclose(host(Hg), Hr, rtol=3e-7)
    if rho > 0 and lam > 0:
        C, G = host(Wg).astype(float).sum(0), host(Hg).astype(float).sum(1)
        np.testing.assert_allclose(rho * C, lam * G, rtol=1e-5)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("frac", FRACS)
def test_reg_cost(dna, shape, frac):
    """kl_cost with weights: eq. (2)."""
    V, W, H = _problem(*shape)
    rho, lam = _weights(W, H, frac)
    got = dna.kl_cost(gpu(V), gpu(W), gpu(H), rho=rho, lam=lam).item()
    ref = oracle.objective(V, W, H, rho, lam)
    assert got == pytest.approx(ref, rel=1e-6)


@pytest.mark.parametrize("frac", FRACS)
@pytest.mark.parametrize("shape", [SHAPES[0], SHAPES[2], (1024, 2300, 64, 0.1, 11)])
def test_reg_iterate_matches_separate_calls(dna, frac, shape):
    """dna_iterate hands each normalisation's sums to the next half-step only
    when they are that step's divisor (not when one weight alone fixes the
    other factor's scale): against the separate entry points, the state after
    two iterations agrees to float32 rounding except at selection ties."""
    V, W, H = _problem(*shape)
    rho, lam = _weights(W, H, frac)
    kw = dict(rho=rho, lam=lam)
    Vg = gpu(V)
    Wa, Ha = gpu(W), gpu(H)
    dna.normalize(0, Wa, Ha, **kw)
    Wb, Hb = Wa.clone(), Ha.clone()
    dna.iterate(Vg, Wa, Ha, 2, **kw)
    for _ in range(2):
        dna.dna_iteration(Vg, Wb, Hb, **kw)
    oa, ob = dna.kl_cost(Vg, Wa, Ha, **kw).item(), dna.kl_cost(Vg, Wb, Hb, **kw).item()
    assert abs(oa - ob) <= 1e-6 * abs(ob)
    for a, b in ((Wa, Wb), (Ha, Hb)):
        a, b = host(a), host(b)
        rel = np.abs(a - b) / np.maximum(np.abs(b), 1e-30)
        assert np.mean(rel > 1e-4) <= 0.01, float(rel.max())


@pytest.mark.parametrize("frac", FRACS)
def test_reg_mu_iterate_matches_separate_calls(dna, frac):
    V, W, H = _problem(*SHAPES[0])
    rho, lam = _weights(W, H, frac)
    kw = dict(rho=rho, lam=lam)
    Vg = gpu(V)
    Wa, Ha = gpu(W), gpu(H)
    dna.normalize(0, Wa, Ha, **kw)
    Wb, Hb = Wa.clone(), Ha.clone()
    dna.mu_iterate(Vg, Wa, Ha, 3, **kw)
    for _ in range(3):
        dna.mu_iteration(Vg, Wb, Hb, **kw)
    assert torch.equal(Wa, Wb) and torch.equal(Ha, Hb)


@pytest.mark.parametrize("frac", FRACS)
@pytest.mark.parametrize("method", ["dna", "mu"])
def test_reg_trajectory(dna, frac, method):
    """20 iterations on a 200 x 300 problem (R = 10): eq. (2) after every
    iteration within 1e-4 of the oracle's; non-increasing when both weights are
    positive (every normalisation is then the penalty-minimising one)."""
    w = synth.config1()
    rho, lam = _weights(w.W, w.H, frac)
    Vg, Wg, Hg = gpu(w.V), gpu(w.W), gpu(w.H)
    obj = host(dna.fit(Vg, Wg, Hg, 20, method=method, record_kl=True, rho=rho, lam=lam))
    fit = oracle.fit_dna if method == "dna" else oracle.fit_mu
    ref = np.array(fit(w.V, w.W, w.H, 20, value_floor=FLOOR32, rho=rho, lam=lam).obj)
    rel = np.abs(obj - ref) / np.abs(ref)
    log_result("reg_trajectory", {"frac": frac, "method": method, "max_rel": float(rel.max()),
                                  "obj_last": float(obj[-1])})
    assert rel.max() <= TRAJ_TOL
    if rho > 0 and lam > 0:
        assert np.all(np.diff(obj) <= 1e-6 * np.abs(obj[:-1]))


def test_reg_zero_weights_unchanged(dna):
    """Weights of exactly zero run the unregularised method bit for bit."""
    V, W, H = _problem(*SHAPES[0])
    Vg = gpu(V)
    Wa, Ha = gpu(W), gpu(H)
    Wb, Hb = Wa.clone(), Ha.clone()
    dna.fit(Vg, Wa, Ha, 3)
    dna.fit(Vg, Wb, Hb, 3, rho=0.0, lam=0.0)
    assert torch.equal(Wa, Wb) and torch.equal(Ha, Hb)


# --------------------------------------------------------------------------- sparse V

SP_SHAPES = [(300, 333, 37, 0.05, 1), (1000, 515, 64, 0.02, 3), (150, 170, 200, 0.08, 6)]


@pytest.mark.parametrize("shape", SP_SHAPES)
@pytest.mark.parametrize("side", [0, 1])
def test_reg_sparse_update(dna, shape, side):
    wk = synth.sparse_problem(*shape)
    V, W, H = wk.V, wk.W, wk.H
    rho, lam = _weights(W, H, FRACS[2])
    sv = dna.SparseV.from_dense(V)
    Wg, Hg = gpu(W), gpu(H)
    if side == 0:
        m = dna.sparse_update_H(sv, Wg, Hg, mask=True, rho=rho, lam=lam)[0]
        got, r = host(Hg), oracle.h_step(V, W, H, value_floor=FLOOR32, lam=lam)
    else:
        m = dna.sparse_update_W(sv, Wg, Hg, mask=True, rho=rho, lam=lam)[0]
        got, r = host(Wg), oracle.w_step(V, W, H, value_floor=FLOOR32, rho=rho)
    ax = 0 if side == 0 else 1
    mask = host(m).astype(bool)
    Wd, Hd = W.astype(float), H.astype(float)
    zgap = recon_gap(Wd @ r.X_mu, Wd @ r.X_newton, 0) if side == 0 else recon_gap(r.X_mu @ Hd, r.X_newton @ Hd, 1)
    rep = selection_report(mask, r.chose_newton, r.margin, r.d_mu, STATE_TIE, zgap)
    same = mask == r.chose_newton
    err = rel_cols(got, r.X, ax)[same]
    assert rep["n_flips_above_tie"] == 0, rep
    assert err.size == 0 or err.max() <= STEP_TOL


def test_reg_sparse_cost_and_trajectory(dna):
    wk = synth.sparse_problem(600, 500, 20, 0.02, 11)
    V, W, H = wk.V, wk.W, wk.H
    rho, lam = _weights(W, H, FRACS[2])
    sv = dna.SparseV.from_dense(V)
    got = dna.sparse_kl_cost(sv, gpu(W), gpu(H), rho=rho, lam=lam).item()
    assert got == pytest.approx(oracle.objective(V, W, H, rho, lam), rel=1e-6)
    obj = host(dna.sparse_fit(sv, gpu(W), gpu(H), 15, record_kl=True, rho=rho, lam=lam))
    ref = np.array(oracle.fit_dna(V, W, H, 15, value_floor=FLOOR32, rho=rho, lam=lam).obj)
    rel = np.abs(obj - ref) / np.abs(ref)
    log_result("reg_sparse_trajectory", {"max_rel": float(rel.max())})
    assert rel.max() <= TRAJ_TOL
    assert np.all(np.diff(obj) <= 1e-6 * np.abs(obj[:-1]))


def test_reg_adjoint_rejects_lambda(dna):
    V, W, H = _problem(40, 30, 4, 0.0, 3)
    with pytest.raises(dna.DNAError) as e:
        dna.unrolled_forward(gpu(V), gpu(W), gpu(H), 2, lam=0.5)
    assert e.value.status == 6
