"""FP64 CPU oracle for the Diagonalized Newton Algorithm (DNA) for KL-divergence NMF.

TEST INFRASTRUCTURE ONLY.  This module is the slow, plain reference that the
HIP path is checked against.  Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import it; the product path never does,
and this module imports nothing from the product package.

Everything is NumPy float64.  Inputs may be float32 arrays: they are upcast, so
an oracle run "from the same state" as the GPU starts from exactly the GPU's
numbers.  Notation follows the paper: V (N x T) data, W (N x R), H (R x T),
Z = W H, eps the gain floor, alpha the step ceiling, rho and lambda the
regularisation weights of eq. (2) (``rho``, ``lam``; 0 in the experiments of
Sec. 4, and 0 by default here).

Readings of the paper that this oracle fixes (each is stated where it is used):

* Newton candidate: eq. (15) for a_r < 0 with the gain floored at eps, and
  eq. (17) for a_r >= 0 with the step capped at alpha*h_r (gain <= 1+alpha).
  Algorithm 1 steps 11 and 24 print the H-product in the wrong place; the
  printed form is not dimensionally consistent, eq. (15)/(17) are.
* Explicit column sums c = W^t 1 (and H 1 in the W step) divide eq. (7) and
  eq. (14), so the step is correct whether or not W was normalised first.
* Zeros of V contribute nothing to Q, Q-bar or the costs (end of Sec. 3).
* Selection: Newton iff d_DNA < d_MU (step 15: ties go to MU).
* Renormalisation eq. (10) with a zero denominator leaves the column at 0.
* Regularisation (eq. 2-5): lambda enters the H step as printed in eq. (7),
  (10), (11) and (14), i.e. every division by c_r becomes one by c_r + lambda;
  the W step is its mirror with g_r + rho.  The selection stays on the
  log-ratio sums of steps 9/14: both candidates satisfy eq. (9), so the rest of
  the regularised per-column cost, sum_r (c_r + lambda) x_r - sum_n v_n, is the
  same (zero) for both.
* Normalisations under regularisation (steps 1, 16, 29).  The printed steps
  (divide by sum + lambda, or + rho) do not give c_r + lambda = 1, which the
  printed step 5 (A = W^t Q - 1) would need, and they change the penalty
  rho sum w + lambda sum h, which is not invariant under moving scale between a
  W column and an H row.  This oracle reads them as: with rho = lambda = 0, the
  paper's unit column sums of W (steps 1, 29) and unit row sums of H (step 16);
  with rho > 0 and lambda > 0, every normalisation applies the scale
  s_r = sqrt(lambda G_r / (rho C_r)) (C = W^t 1, G = H 1) to W column r and
  1/s_r to H row r, the scale that minimises the penalty with W H fixed (after
  it rho C_r = lambda G_r), so no normalisation raises eq. (2); with one weight
  zero, eq. (2) has no minimiser unless the unpenalised factor's scale is fixed,
  so every normalisation sets that factor to unit sums (W columns when only
  lambda > 0, H rows when only rho > 0).
* ``value_floor`` (default 0: the paper's method on the positive reals): when
  positive, both candidates are raised to at least this value after the
  renormalisation.  In exact arithmetic no update maps a positive entry to 0
  (the floor eps bounds the shrink per step), but a floating-point format
  underflows an entry that keeps shrinking, and 0 is a fixed point of every
  update; passing the smallest positive normal number of the storage format
  (float32: 2**-126) keeps the run on the positive reals that format can hold.

Functions with no independent pin are marked "parity unpinned" in their
docstring; at present there are none (the pins live in tests/).
"""
from __future__ import annotations

import dataclasses

import numpy as np

EPS = 0.01    # Sec. 4: gain floor epsilon
ALPHA = 4.0   # Sec. 4: step ceiling alpha


class DomainError(ValueError):
    """Input outside the method's domain (zero W column sum, z = 0 where v > 0, ...)."""


def _f64(x):
    return np.asarray(x, dtype=np.float64)


# ---------------------------------------------------------------------------
# Costs (eq. 1; Algorithm 1 steps 9, 14, 22, 27)
# ---------------------------------------------------------------------------

def kl_divergence(V, Z):
    """Eq. (1): sum v log(v/z) - sum v + sum z, with v = 0 terms of the log sum
    left out (end of Sec. 3).  +inf if some z <= 0 where v > 0."""
    V, Z = _f64(V), _f64(Z)
    pos = V > 0
    if np.any(Z[pos] <= 0):
        return np.inf
    return float(np.sum(V[pos] * np.log(V[pos] / Z[pos])) - V.sum() + Z.sum())


def kl_cost(V, W, H):
    """Eq. (1) at Z = W H."""
    return kl_divergence(V, _f64(W) @ _f64(H))


def objective(V, W, H, rho=0.0, lam=0.0):
    """Eq. (2): d_KL(V, W H) + rho sum w + lambda sum h."""
    W, H = _f64(W), _f64(H)
    return kl_cost(V, W, H) + rho * float(W.sum()) + lam * float(H.sum())


def partial_cost(V, Z, axis=0):
    """Steps 9/14 (axis=0, one value per column) and 22/27 (axis=1, per row):
    sum over the other index of v log(v/z) for v > 0.  A column (row) with
    z <= 0 at some v > 0 costs +inf."""
    V, Z = _f64(V), _f64(Z)
    pos = V > 0
    bad = pos & (Z <= 0)
    term = np.zeros_like(V)
    ok = pos & ~bad
    term[ok] = V[ok] * np.log(V[ok] / Z[ok])
    d = term.sum(axis=axis)
    d[bad.any(axis=axis)] = np.inf
    return d


# ---------------------------------------------------------------------------
# Building blocks of one half-step (Sec. 2)
# ---------------------------------------------------------------------------

def ratios(V, Z):
    """Q = V / Z and Q-bar = V / (Z*Z) (steps 3 and 10), zero where v = 0.
    z <= 0 at v > 0 is outside the domain."""
    V, Z = _f64(V), _f64(Z)
    pos = V > 0
    if np.any(Z[pos] <= 0):
        raise DomainError("z <= 0 where v > 0")
    Q = np.zeros_like(V)
    Qb = np.zeros_like(V)
    Q[pos] = V[pos] / Z[pos]
    Qb[pos] = V[pos] / (Z[pos] * Z[pos])
    return Q, Qb


def newton_candidate(X, A, B, eps=EPS, alpha=ALPHA):
    """Element-wise diagonal Newton update before renormalisation.

    a < 0 : x * max(x b / (x b - a), eps)      eq. (15), gain floored (Sec. 2.3)
    a >= 0: x + min(a / b, alpha * x)          eq. (17), step capped (Sec. 2.3)

    For a >= 0 and b = 0 the step a/b is +inf (a > 0) or 0 (a = 0), so the cap
    decides.  x = 0 maps to 0 in both branches (fixed point, Sec. 2.2).
    """
    X, A, B = _f64(X), _f64(A), _f64(B)
    out = np.empty_like(X)
    neg = A < 0
    xb = X[neg] * B[neg]
    gain = xb / (xb - A[neg])          # denominator > 0 because a < 0 <= x b
    out[neg] = X[neg] * np.maximum(gain, eps)
    pos = ~neg
    a, b, x = A[pos], B[pos], X[pos]
    step = np.where(b > 0, a / np.where(b > 0, b, 1.0),
                    np.where(a > 0, np.inf, 0.0))
    out[pos] = x + np.minimum(step, alpha * x)
    return out


def renormalize(X, c, s, axis=0):
    """Eq. (10): scale each column (axis=0) or row (axis=1) of X so that
    sum_r c_r x_r equals s (the data sum of that column / row); the caller
    passes c_r = (W^t 1)_r + lambda (H step) or (H 1)_r + rho (W step).  A zero
    denominator leaves the column (row) unchanged (it is all zero)."""
    X = _f64(X)
    if axis == 0:
        den = c @ X
        f = np.divide(s, den, out=np.ones_like(den), where=den > 0)
        return X * f[None, :]
    den = X @ c
    f = np.divide(s, den, out=np.ones_like(den), where=den > 0)
    return X * f[:, None]


@dataclasses.dataclass
class StepResult:
    """Result of one half-step.  ``X`` is the updated factor (H or W)."""
    X: np.ndarray
    chose_newton: np.ndarray
    d_sel: np.ndarray
    d_mu: np.ndarray
    d_newton: np.ndarray
    margin: np.ndarray          # d_mu - d_newton
    A: np.ndarray
    B: np.ndarray
    X_mu: np.ndarray
    X_newton: np.ndarray


def _select(d_mu, d_nr, X_mu, X_nr, axis):
    """Step 15 / 28: Newton where d_DNA < d_MU, MU otherwise (ties -> MU)."""
    choose = d_nr < d_mu
    if axis == 0:
        X = np.where(choose[None, :], X_nr, X_mu)
    else:
        X = np.where(choose[:, None], X_nr, X_mu)
    d_sel = np.where(choose, d_nr, d_mu)
    with np.errstate(invalid="ignore"):
        margin = d_mu - d_nr
    return choose, X, d_sel, margin


def _select_newton_first(d_cur, d_nr, X, X_mu, X_nr, c, s, axis):
    """The damped selection (reading of Sec. 5's "more refined step damping"):
    evaluate the Newton candidate only and keep it iff it does not raise the
    column's (axis 0) or row's (axis 1) objective of eq. (5),
        d + sum_r c_r x_r - sum v       (c including lambda, resp. rho),
    above the current state's; else take the MU candidate, which never raises
    it (Sec. 2.1), without evaluating its cost.  Returns choose, X, d_sel (NaN
    where MU is kept: its cost is not formed), margin = objective(current) -
    objective(Newton)."""
    if axis == 0:
        obj_cur = d_cur + c @ X - s
        obj_nr = d_nr + c @ X_nr - s
    else:
        obj_cur = d_cur + X @ c - s
        obj_nr = d_nr + X_nr @ c - s
    with np.errstate(invalid="ignore"):
        margin = obj_cur - obj_nr
    choose = np.isfinite(d_nr) & (obj_nr <= obj_cur)
    if axis == 0:
        Xo = np.where(choose[None, :], X_nr, X_mu)
    else:
        Xo = np.where(choose[:, None], X_nr, X_mu)
    d_sel = np.where(choose, d_nr, np.nan)
    return choose, Xo, d_sel, margin


def h_step(V, W, H, eps=EPS, alpha=ALPHA, value_floor=0.0, lam=0.0, select="both"):
    """One DNA update of H with W fixed: Algorithm 1 steps 4-15 (Sec. 2-3).

    c = W^t 1 + lambda; Z = W H; Q, Q-bar (steps 2-3, 10); A = W^t Q / c - 1
    (eq. 7, step 5); B = (W*W)^t Q-bar / c (eq. 14, step 10); MU candidate
    H(1+A) (eq. 11, step 6); Newton candidate (eq. 15/17, step 11)
    renormalised by eq. (10) with s = 1^t V; per-column costs (steps 7-9,
    12-14); selection (step 15).  ``lam`` is the H weight of eq. (2).

    ``select="newton_first"``: the damped selection of _select_newton_first in
    place of steps 7-9 and 15 (the MU candidate's cost is not evaluated;
    ``d_mu`` is then NaN).
    """
    V, W, H = _f64(V), _f64(W), _f64(H)
    c = W.sum(axis=0)
    if np.any(c <= 0):
        raise DomainError("a column of W sums to zero")
    c = c + lam
    Q, Qb = ratios(V, W @ H)
    A = (W.T @ Q) / c[:, None] - 1.0
    B = ((W * W).T @ Qb) / c[:, None]
    H_mu = np.maximum(H * (1.0 + A), value_floor)
    H_nr = np.maximum(renormalize(newton_candidate(H, A, B, eps, alpha), c, V.sum(axis=0), axis=0),
                      value_floor)
    d_nr = partial_cost(V, W @ H_nr, axis=0)
    if select == "newton_first":
        d_cur = partial_cost(V, W @ H, axis=0)
        choose, X, d_sel, margin = _select_newton_first(d_cur, d_nr, H, H_mu, H_nr, c, V.sum(axis=0), 0)
        return StepResult(X, choose, d_sel, np.full_like(d_nr, np.nan), d_nr, margin, A, B, H_mu, H_nr)
    d_mu = partial_cost(V, W @ H_mu, axis=0)
    choose, X, d_sel, margin = _select(d_mu, d_nr, H_mu, H_nr, axis=0)
    return StepResult(X, choose, d_sel, d_mu, d_nr, margin, A, B, H_mu, H_nr)


def w_step(V, W, H, eps=EPS, alpha=ALPHA, value_floor=0.0, rho=0.0, select="both"):
    """One DNA update of W with H fixed: Algorithm 1 steps 17-28.

    The mirror of ``h_step`` written out directly: g = H 1 + rho;
    A = Q H^t / g - 1 (step 18); B = Q-bar (H*H)^t / g (step 23); MU candidate
    W(1+A) (step 19); Newton candidate (step 24 read as eq. 15/17) with each
    row renormalised so that sum_r g_r w_nr = (V 1)_n; per-row costs
    (steps 20-22, 25-27); selection per row (step 28).  ``rho`` is the W weight
    of eq. (2).  ``select`` as in ``h_step``, per row.
    """
    V, W, H = _f64(V), _f64(W), _f64(H)
    g = H.sum(axis=1)
    if np.any(g <= 0):
        raise DomainError("a row of H sums to zero")
    g = g + rho
    Q, Qb = ratios(V, W @ H)
    A = (Q @ H.T) / g[None, :] - 1.0
    B = (Qb @ (H * H).T) / g[None, :]
    W_mu = np.maximum(W * (1.0 + A), value_floor)
    W_nr = np.maximum(renormalize(newton_candidate(W, A, B, eps, alpha), g, V.sum(axis=1), axis=1),
                      value_floor)
    d_nr = partial_cost(V, W_nr @ H, axis=1)
    if select == "newton_first":
        d_cur = partial_cost(V, W @ H, axis=1)
        choose, X, d_sel, margin = _select_newton_first(d_cur, d_nr, W, W_mu, W_nr, g, V.sum(axis=1), 1)
        return StepResult(X, choose, d_sel, np.full_like(d_nr, np.nan), d_nr, margin, A, B, W_mu, W_nr)
    d_mu = partial_cost(V, W_mu @ H, axis=1)
    choose, X, d_sel, margin = _select(d_mu, d_nr, W_mu, W_nr, axis=1)
    return StepResult(X, choose, d_sel, d_mu, d_nr, margin, A, B, W_mu, W_nr)


def mu_h_step(V, W, H, value_floor=0.0, lam=0.0):
    """Plain MU update of H (eq. 11; Lee-Seung at lambda = 0):
    H <- H * (W^t Q) / (W^t 1 + lambda).  Also returns the per-column partial
    cost sum_{v>0} v log(v/z) of the INPUT state (the cost that "MU with cost"
    monitors, computed from the same Z)."""
    V, W, H = _f64(V), _f64(W), _f64(H)
    c = W.sum(axis=0)
    if np.any(c <= 0):
        raise DomainError("a column of W sums to zero")
    c = c + lam
    Z = W @ H
    Q, _ = ratios(V, Z)
    return np.maximum(H * (W.T @ Q) / c[:, None], value_floor), partial_cost(V, Z, axis=0)


def mu_w_step(V, W, H, value_floor=0.0, rho=0.0):
    """Plain MU update of W: W <- W * (Q H^t) / (H 1 + rho); per-row input cost."""
    V, W, H = _f64(V), _f64(W), _f64(H)
    g = H.sum(axis=1)
    if np.any(g <= 0):
        raise DomainError("a row of H sums to zero")
    g = g + rho
    Z = W @ H
    Q, _ = ratios(V, Z)
    return np.maximum(W * (Q @ H.T) / g[None, :], value_floor), partial_cost(V, Z, axis=1)


# ---------------------------------------------------------------------------
# Normalisations (Algorithm 1 steps 1, 16, 29) and full runs
# ---------------------------------------------------------------------------

def normalize_w_columns(W, H):
    """Steps 1 and 29 at lambda = 0: divide column r of W by its sum and
    multiply row r of H by the same number (W H is unchanged)."""
    W, H = _f64(W), _f64(H)
    c = W.sum(axis=0)
    if np.any(c <= 0):
        raise DomainError("a column of W sums to zero")
    return W / c[None, :], H * c[:, None]


def normalize_h_rows(W, H):
    """Step 16 at rho = 0: divide row r of H by its sum sum_t h_rt and multiply
    column r of W by the same number."""
    W, H = _f64(W), _f64(H)
    g = H.sum(axis=1)
    if np.any(g <= 0):
        raise DomainError("a row of H sums to zero")
    return W * g[None, :], H / g[:, None]


def normalize(W, H, side, rho=0.0, lam=0.0):
    """Steps 1 and 29 (side 0) and step 16 (side 1) under the regularisation
    weights of eq. (2), in the reading stated in the module header:

    rho = lambda = 0  side 0: unit W column sums; side 1: unit H row sums
    rho > 0, lambda > 0  either side: W column r times s_r, H row r divided by
                      s_r, s_r = sqrt(lambda G_r / (rho C_r)) (C = W^t 1,
                      G = H 1), the scale minimising rho C_r s + lambda G_r / s
    lambda > 0 only   either side: unit W column sums
    rho > 0 only      either side: unit H row sums

    W H is unchanged in every case."""
    if rho < 0 or lam < 0:
        raise ValueError("rho and lambda must be >= 0")
    if rho > 0 and lam > 0:
        W, H = _f64(W), _f64(H)
        C, G = W.sum(axis=0), H.sum(axis=1)
        if np.any(C <= 0) or np.any(G <= 0):
            raise DomainError("a column of W or a row of H sums to zero")
        s = np.sqrt(lam * G / (rho * C))
        return W * s[None, :], H / s[:, None]
    if lam > 0:
        side = 0
    elif rho > 0:
        side = 1
    return normalize_w_columns(W, H) if side == 0 else normalize_h_rows(W, H)


_normalize = normalize      # fit_mu's ``normalize`` argument shadows the name


@dataclasses.dataclass
class FitResult:
    W: np.ndarray
    H: np.ndarray
    kl: list                  # eq. (1) after every full iteration (index 0 = start)
    newton_frac_h: list       # fraction of columns taking Newton, per iteration
    newton_frac_w: list       # fraction of rows taking Newton, per iteration
    obj: list = dataclasses.field(default_factory=list)   # eq. (2), same points as kl


def fit_dna(V, W, H, iters, eps=EPS, alpha=ALPHA, value_floor=0.0, rho=0.0, lam=0.0, select="both"):
    """Algorithm 1: step 1, then per iteration H half-step (4-15), step 16,
    W half-step (17-28), step 29.  Z and Q are recomputed from W H at the start
    of each half-step, which equals carrying them because the normalisations
    leave W H unchanged.  ``select`` as in ``h_step``."""
    V = _f64(V)
    W, H = normalize(W, H, 0, rho, lam)
    kl = [kl_cost(V, W, H)]
    obj = [objective(V, W, H, rho, lam)]
    fh, fw = [], []
    for _ in range(iters):
        r = h_step(V, W, H, eps, alpha, value_floor, lam=lam, select=select)
        H = r.X
        fh.append(float(r.chose_newton.mean()))
        W, H = normalize(W, H, 1, rho, lam)
        r = w_step(V, W, H, eps, alpha, value_floor, rho=rho, select=select)
        W = r.X
        fw.append(float(r.chose_newton.mean()))
        W, H = normalize(W, H, 0, rho, lam)
        kl.append(kl_cost(V, W, H))
        obj.append(objective(V, W, H, rho, lam))
    return FitResult(W, H, kl, fh, fw, obj)


def fit_mu(V, W, H, iters, normalize=True, value_floor=0.0, rho=0.0, lam=0.0):
    """MU reference: Algorithm 1 with only the MU-labelled steps.  With
    ``normalize=False`` it is textbook Lee-Seung MU without steps 1/16/29."""
    V = _f64(V)
    W, H = _f64(W), _f64(H)
    if normalize:
        W, H = _normalize(W, H, 0, rho, lam)
    kl = [kl_cost(V, W, H)]
    obj = [objective(V, W, H, rho, lam)]
    for _ in range(iters):
        H, _ = mu_h_step(V, W, H, value_floor, lam=lam)
        if normalize:
            W, H = _normalize(W, H, 1, rho, lam)
        W, _ = mu_w_step(V, W, H, value_floor, rho=rho)
        if normalize:
            W, H = _normalize(W, H, 0, rho, lam)
        kl.append(kl_cost(V, W, H))
        obj.append(objective(V, W, H, rho, lam))
    return FitResult(W, H, kl, [], [], obj)


def unrolled_h(V, W, H_init, K, eps=EPS, alpha=ALPHA, value_floor=0.0):
    """K DNA H-updates with W fixed (no normalisation between them).

    Returns the list [H_0 .. H_K] and the K selection masks.  This is the
    forward pass of the differentiable unrolled H-solve."""
    Hs = [_f64(H_init)]
    masks = []
    for _ in range(K):
        r = h_step(V, W, Hs[-1], eps, alpha, value_floor)
        Hs.append(r.X)
        masks.append(r.chose_newton)
    return Hs, masks
