"""Shared helpers for the GPU parity tests (comparison norms, transfers, logging)."""
import json
import os

import numpy as np
import torch

# Measured errors of each parity test are appended as JSON lines to the file
# named by DNA_PARITY_LOG (nothing is logged when it is unset).
LOG_PATH = os.environ.get("DNA_PARITY_LOG")

# Per-step tolerance in FP32 (from identical states): max-norm per column (row)
# relative to the oracle's max-norm of that column (row).
STEP_TOL = 1e-5
# Trajectory tolerance: relative KL after every iteration.
TRAJ_TOL = 1e-4
# Selection from identical candidates (oracle re-scores the GPU's candidates in
# float64): every column with |d_MU - d_DNA| / |d_MU| above this must agree.
SELECT_TIE = 1e-12
# Selection from an identical state (both sides form their own candidates, the
# GPU in float32).  Two checks, both at the 1e-12 tie bound: (1) every GPU
# decision equals the FP64 re-scoring of the GPU's own candidates (``rescore``)
# wherever that margin exceeds 1e-12 relative; (2) against the oracle's own
# decisions, flips are allowed only at the oracle's relative margins <= 1e-12,
# or where both candidates reconstruct the same Z (Z_TIE).  The float32
# candidates differ from the oracle's by about 1e-7 relative, which could in
# principle move a margin of that size; every measured flip so far is an exact
# tie (R = 1: margins <= 6e-16) or a Z_TIE case (N = 1, T = 1), so the bound is
# kept at 1e-12.
STATE_TIE = 1e-12


EPS32 = 2.0 ** -24
# Smallest positive normal float32: the factors' storage format.  The oracle is
# run with this value floor wherever it is compared with the float32 path.
FLOOR32 = float(np.finfo(np.float32).tiny)


def cost_err(d_gpu, d_ref, vsum):
    """max over columns of |d_gpu - d_ref| / (|d_ref| + 8 eps32 sum v / STEP_TOL).

    A cost sum_{v>0} v log(v/z) evaluated from float32 reconstructions carries an
    absolute error of a few float32 ulps of each log, i.e. about eps32 * sum v,
    whatever the size of the cost itself (which may be ~0 when z fits v); the
    floor keeps the comparison relative where d is large and absolute where it
    vanishes.  <= 1 means within STEP_TOL."""
    d_gpu, d_ref, vsum = (np.asarray(x, float) for x in (d_gpu, d_ref, vsum))
    den = STEP_TOL * np.abs(d_ref) + 8 * EPS32 * vsum
    return float(np.max(np.abs(d_gpu - d_ref) / np.maximum(den, 1e-300))) if d_ref.size else 0.0


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, dtype=np.float32))).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel_cols(got, ref, axis=0):
    """max over columns (axis=0) or rows (axis=1) of ||got-ref||_inf / ||ref||_inf."""
    got, ref = np.asarray(got, float), np.asarray(ref, float)
    num = np.max(np.abs(got - ref), axis=axis)
    den = np.max(np.abs(ref), axis=axis)
    den = np.where(den > 0, den, 1.0)
    return num / den


def log_result(name, payload):
    if not LOG_PATH:
        return
    os.makedirs(os.path.dirname(os.path.abspath(LOG_PATH)), exist_ok=True)
    with open(LOG_PATH, "a") as f:
        f.write(json.dumps({"test": name, **payload}) + "\n")


# Two candidates whose reconstructions agree to this relative precision at every
# data entry are the same point to float32 resolution: their costs tie whatever
# their size (e.g. N = 1, where both reproduce v exactly, or R = 1).
Z_TIE = 1e-6


def recon_gap(Z_mu, Z_newton, axis):
    """max over the data entries of a column (axis=0) / row (axis=1) of
    |z_MU - z_DNA| / max(z_MU, z_DNA)."""
    Z_mu, Z_newton = np.asarray(Z_mu, float), np.asarray(Z_newton, float)
    den = np.maximum(np.maximum(np.abs(Z_mu), np.abs(Z_newton)), 1e-300)
    return np.max(np.abs(Z_mu - Z_newton) / den, axis=axis)


def selection_report(mask_gpu, mask_ref, margin_ref, d_mu_ref, tie, zgap=None):
    """Flips between two selections, each with the oracle's relative margin.  A
    flip is a tie (allowed) when |margin| <= tie * |d_MU| or, given ``zgap``, when
    the two candidates reconstruct the same Z to within Z_TIE."""
    mask_gpu = np.asarray(mask_gpu).astype(bool)
    mask_ref = np.asarray(mask_ref).astype(bool)
    with np.errstate(invalid="ignore", divide="ignore"):
        rel = np.abs(margin_ref) / np.maximum(np.abs(d_mu_ref), 1e-300)
    if zgap is None:
        zgap = np.full(mask_ref.shape, np.inf)
    flips = np.nonzero(mask_gpu != mask_ref)[0]
    bad = [int(i) for i in flips if not (rel[i] <= tie or zgap[i] <= Z_TIE)]
    return {
        "n": int(mask_ref.size),
        "newton_frac": float(mask_ref.mean()) if mask_ref.size else 0.0,
        "flips": int(flips.size),
        "flip_margins": [float(rel[i]) for i in flips[:20]],
        "flips_above_tie": bad[:20],
        "n_flips_above_tie": len(bad),
    }


def rescore(V, F, Xmu, Xn, side):
    """FP64 re-scoring of a pair of candidates (the GPU's own): the step 9 / 14
    costs per column (side 0, F = W) or row (side 1, F = H), the choice
    (Newton iff d_DNA < d_MU), the margin and the reconstruction gap."""
    from oracle import dna_oracle as O
    V = np.asarray(V, float)
    F = np.asarray(F, float)
    Xmu, Xn = np.asarray(Xmu, float), np.asarray(Xn, float)
    if side == 0:
        Zm, Zn = F @ Xmu, F @ Xn
    else:
        Zm, Zn = Xmu @ F, Xn @ F
    ax = 0 if side == 0 else 1
    d_mu, d_n = O.partial_cost(V, Zm, ax), O.partial_cost(V, Zn, ax)
    return d_n < d_mu, d_mu - d_n, d_mu, recon_gap(Zm, Zn, ax)
