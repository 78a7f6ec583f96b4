"""GPU accuracy of the 16-bit precision forms (BF16 / FP16 matrix-product operands,
float32 accumulation, float64 selection and cost sums) against the FP64 oracle.

The forms are not the method of the paper at another precision: every product
operand is rounded to 16 bits, so the comparison with the FP64 oracle has an
error bound set by the operand format, not the 1e-5 of the float32 path.
Rounding an operand costs a relative error of at most u (BF16: u = 2^-8, FP16:
u = 2^-11).  Z = W H and the gradient sums are sums of non-negative terms, so
each carries a relative error of at most 2u (both operands rounded) plus one
more u for the rounded ratio; the candidates are formed from those sums in
float32.  The asserted bounds below are these first-order bounds with a factor
of two of headroom for the Newton quotient a / b; the measured errors are
logged beside them.  Selections may differ from the oracle's only where the
oracle's relative margin is below the same order, the resolution of a cost
computed from 16-bit reconstructions.

The bounds: gradient sums 4u, one step 4u, selection ties 2u (measured: about
1u, 1u and at most 0.7u), KL trajectories u.  The trajectory bound holds only
because the ratio pass forms Z with the updated factor split into two 16-bit
parts (BF16: both factors): with a single rounding of H, the gradient is taken
a relative u away from the point the step is applied to, and the trajectory
drifts by 15% (BF16) / 1.3% (FP16) of the KL within 20 iterations."""
import numpy as np
import pytest
import torch

import oracle
from paper_1301_3389_amd import synth
from parity_util import FLOOR32, gpu, host, log_result, recon_gap, rel_cols, selection_report

pytestmark = pytest.mark.gpu

UNIT = {"bf16": 2.0 ** -8, "fp16": 2.0 ** -11}


def step_tol(gemm):
    return 4 * UNIT[gemm]


def tie_tol(gemm):
    return 2 * UNIT[gemm]


def traj_tol(gemm):
    return UNIT[gemm]


SHAPES = [
    # N, T, R, zero_frac, seed
    (300, 333, 37, 0.2, 1),
    (257, 130, 10, 0.0, 2),
    (1000, 515, 64, 0.1, 4),
    (130, 200, 1, 0.0, 5),
    (200, 300, 129, 0.05, 9),
    # T % 4 == 0 with ragged N and several K tiles: the W step's transposed
    # tiles read V in 16-byte pieces
    (300, 516, 40, 0.1, 11),
]


def _problem(N, T, R, zf, seed):
    w = synth.random_problem(N, T, R, seed, zero_frac=zf)
    V = w.V.copy()
    V[0, :] = np.maximum(V[0, :], 1.0)
    V[:, 0] = np.maximum(V[:, 0], 1.0)
    return V, w.W, w.H


def _rel_gain_err(A, A_ref):
    # A = g - 1 with g = u / c the MU gain: compare through g
    return float(np.max(np.abs(A - A_ref) / (np.abs(1.0 + A_ref) + 1e-30)))


@pytest.mark.parametrize("gemm", ["bf16", "fp16"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("side", [0, 1])
def test_gradient_hessian_16(dna, gemm, shape, side):
    V, W, H = _problem(*shape)
    A, B = dna.gradient_hessian(side, gpu(V), gpu(W), gpu(H), gemm=gemm)
    r = (oracle.h_step if side == 0 else oracle.w_step)(V, W, H, value_floor=FLOOR32)
    errA = _rel_gain_err(host(A), r.A)
    errB = float(rel_cols(host(B), r.B, axis=0 if side == 0 else 1).max())
    log_result("precision_gradient_hessian", {"gemm": gemm, "shape": shape, "side": side,
                                              "errA": errA, "errB": errB, "unit": UNIT[gemm]})
    assert errA <= 4 * UNIT[gemm]
    assert errB <= 4 * UNIT[gemm]


def _step_report(dna, V, W, H, side, gemm, cols=None, rows=None):
    """One 16-bit half-step on the GPU against the oracle's float64 step from the
    same float32 state, on all or on sampled columns (H) / rows (W)."""
    Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
    if side == 0:
        X = Hg.clone()
        m, _, _ = dna.update_H(Vg, Wg, X, mask=True, d_sel=True, margin=True, gemm=gemm)
        sel = slice(None) if cols is None else cols
        r = oracle.h_step(V[:, sel], W, H[:, sel], value_floor=FLOOR32)
        got = host(X)[:, sel]
        mask = host(m)[sel].astype(bool)
        Wd = W.astype(float)
        zg = recon_gap(Wd @ r.X_mu, Wd @ r.X_newton, 0)
        ax = 0
    else:
        X = Wg.clone()
        m, _, _ = dna.update_W(Vg, X, Hg, mask=True, d_sel=True, margin=True, gemm=gemm)
        sel = slice(None) if rows is None else rows
        r = oracle.w_step(V[sel], W[sel], H, value_floor=FLOOR32)
        got = host(X)[sel]
        mask = host(m)[sel].astype(bool)
        Hd = H.astype(float)
        zg = recon_gap(r.X_mu @ Hd, r.X_newton @ Hd, 1)
        ax = 1
    rep = selection_report(mask, r.chose_newton, r.margin, r.d_mu, tie_tol(gemm), zg)
    same = mask == r.chose_newton
    err = rel_cols(got, r.X, ax)[same]
    return rep, err


@pytest.mark.parametrize("gemm", ["bf16", "fp16"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("side", [0, 1])
def test_update_16(dna, gemm, shape, side):
    V, W, H = _problem(*shape)
    rep, err = _step_report(dna, V, W, H, side, gemm)
    e = float(err.max()) if err.size else 0.0
    log_result("precision_update", {"gemm": gemm, "shape": shape, "side": side, "sel": rep, "err": e,
                                    "err_median": float(np.median(err)) if err.size else 0.0,
                                    "bound": step_tol(gemm)})
    assert rep["n_flips_above_tie"] == 0
    assert e <= step_tol(gemm)


@pytest.mark.parametrize("gemm", ["bf16", "fp16"])
def test_trajectory_16_config1(dna, gemm):
    """20 alternating DNA iterations in the 16-bit form: the KL after each one
    follows the FP64 oracle's trajectory to the accuracy of the form."""
    w = synth.config(1)
    Vg, Wg, Hg = gpu(w.V), gpu(w.W), gpu(w.H)
    kl_ref = np.array(oracle.fit_dna(w.V, w.W, w.H, iters=20, value_floor=FLOOR32).kl)
    kl = host(dna.fit(Vg, Wg, Hg, 20, method="dna", record_kl=True, gemm=gemm))
    rel = np.abs(kl - kl_ref) / np.abs(kl_ref)
    log_result("precision_trajectory_config1", {"gemm": gemm, "rel": rel.tolist(), "kl": kl.tolist(),
                                                "kl_ref": kl_ref.tolist()})
    assert rel.max() <= traj_tol(gemm)


def test_trajectory_fp16_one_call(dna):
    """20 DNA iterations in FP16 as one native call, in which each cost pass
    bounds the next Z pass's Q maxima (no maxima pass after the first half
    step): the final KL follows the FP64 oracle's to the form's accuracy, and
    matches the iteration-by-iteration run (a maxima pass every half step) to
    within the same bound."""
    w = synth.config(1)
    kl_ref = oracle.fit_dna(w.V, w.W, w.H, iters=20, value_floor=FLOOR32).kl[-1]
    Vg, Wg, Hg = gpu(w.V), gpu(w.W), gpu(w.H)
    dna.fit(Vg, Wg, Hg, 20, method="dna", gemm="fp16")
    kl_one = float(host(dna.kl_cost(Vg, Wg, Hg))[0])
    Vg, Wg, Hg = gpu(w.V), gpu(w.W), gpu(w.H)
    for _ in range(20):
        dna.fit(Vg, Wg, Hg, 1, method="dna", gemm="fp16")
    kl_each = float(host(dna.kl_cost(Vg, Wg, Hg))[0])
    log_result("precision_trajectory_fp16_one_call", {"kl_one": kl_one, "kl_each": kl_each, "kl_ref": kl_ref})
    assert abs(kl_one - kl_ref) / abs(kl_ref) <= traj_tol("fp16")
    assert abs(kl_one - kl_each) / abs(kl_each) <= traj_tol("fp16")


_WORKLOADS = {}


def _workload(k):
    if k not in _WORKLOADS:
        _WORKLOADS.clear()
        _WORKLOADS[k] = synth.config(k)
    return _WORKLOADS[k]


@pytest.mark.parametrize("k,gemm", [(3, "bf16"), (3, "fp16"), (4, "fp16"), (4, "bf16")])
def test_full_size_sampled_16(dna, k, gemm):
    """A full-size H step and W step in the 16-bit form, checked on 0.1% (at
    least 24) sampled columns and rows against the oracle."""
    w = _workload(k)
    N, T = w.V.shape
    rng = np.random.default_rng(100 + k)
    cols = np.sort(rng.choice(T, size=max(24, T // 1000), replace=False))
    rows = np.sort(rng.choice(N, size=max(24, N // 1000), replace=False))
    out = {}
    for side in (0, 1):
        rep, err = _step_report(dna, w.V, w.W, w.H, side, gemm, cols=cols, rows=rows)
        e = float(err.max()) if err.size else 0.0
        out[side] = (rep, e)
        log_result("precision_full_size_sampled", {"config": k, "gemm": gemm, "side": side, "sel": rep,
                                                   "err": e, "err_median": float(np.median(err)) if err.size
                                                   else 0.0, "bound": step_tol(gemm)})
    torch.cuda.empty_cache()
    for side in (0, 1):
        rep, e = out[side]
        assert rep["n_flips_above_tie"] == 0
        assert e <= step_tol(gemm)
