"""Reference gradient of K unrolled DNA H-updates (W fixed), FP64 on the CPU.

TEST INFRASTRUCTURE ONLY (see dna_oracle.py): imported by tests and the
benchmark's CPU-baseline leg, never by the product path.

The forward H-update (Algorithm 1 steps 4-15, read as in dna_oracle.h_step) is
transcribed into float64 PyTorch CPU operations and differentiated by autograd.
The per-column MU/Newton selection of every update is frozen: it is taken from
the NumPy oracle's own forward pass unless the caller supplies the masks.  The
inner branches (a < 0 or a >= 0, eps floor, alpha cap) are evaluated inside the
transcription, so autograd follows the branch that is active at each entry.

Domain of the gradient: z = (W H)_nt > 0 everywhere (true when W > 0 and every
H column has a positive entry).  Q = V/Z and Q-bar = V/Z^2 are then smooth in
V, so at entries with v = 0 the gradient with respect to v is the derivative
of those rational expressions; it is what a one-sided finite difference gives.
"""
from __future__ import annotations

import numpy as np
import torch

from .dna_oracle import ALPHA, EPS, unrolled_h


def h_update_torch(V, W, H, chose_newton, eps=EPS, alpha=ALPHA, value_floor=0.0, perturb=None):
    """One H-update as torch float64 ops, selection given by ``chose_newton``.
    ``value_floor`` as in dna_oracle.h_step (clamped entries carry no gradient).

    ``perturb`` (default None: the update itself) is a sensitivity probe for
    judging float32 results, not part of the method: a pair (nA, nB) of R x T
    arrays of relative perturbations applied to the MU gain 1 + A and to B after
    eq. (7) and eq. (14), with every branch (sign of a, eps floor, alpha cap)
    decided on the unperturbed values, so that the result moves smoothly; or a
    triple (nA, nB, True): the same perturbations applied before the branches
    are decided, so that they may also move an entry across a branch
    boundary, as a float32 evaluation of A and B can."""
    c = W.sum(dim=0)
    Z = W @ H
    Q = V / Z
    Qb = V / (Z * Z)
    A = (W.t() @ Q) / c[:, None] - 1.0                 # eq. (7)
    B = ((W * W).t() @ Qb) / c[:, None]                # eq. (14)
    if perturb is not None and len(perturb) > 2 and perturb[2]:
        nA, nB = (torch.as_tensor(np.asarray(x, dtype=np.float64)) for x in perturb[:2])
        A = A + nA * (1.0 + A).detach()
        B = B * (1.0 + nB)
        perturb = None
    ones = torch.ones_like(H)
    neg = (A < 0).detach()
    b_ok = (B > 0).detach()
    hb = (H * B).detach()
    floor = neg & (hb / torch.where(neg, hb - A.detach(), ones) < eps)
    step0 = A.detach() / torch.where(b_ok & ~neg, B.detach(), ones)
    cap = (~neg) & (((~b_ok) & (A > 0).detach()) | (b_ok & (step0 > alpha * H.detach())))
    if perturb is not None:
        nA, nB = (torch.as_tensor(np.asarray(x, dtype=np.float64)) for x in perturb[:2])
        A = A + nA * (1.0 + A).detach()
        B = B * (1.0 + nB)
    H_mu = H * (1.0 + A)                               # eq. (11)
    hb = H * B
    gain = hb / torch.where(neg, hb - A, ones)          # eq. (15) gain, a < 0
    h_neg = torch.where(floor, eps * H, H * gain)
    step = A / torch.where(b_ok & ~neg, B, ones)        # eq. (17) step, a >= 0
    h_pos = torch.where(cap, (1.0 + alpha) * H, H + torch.where(b_ok, step, torch.zeros_like(step)))
    Hn = torch.where(neg, h_neg, h_pos)
    s = V.sum(dim=0)
    den = (c[:, None] * Hn).sum(dim=0)                  # eq. (10) denominator
    Hn = Hn * (s / den)[None, :]
    if value_floor > 0:
        Hn = torch.clamp(Hn, min=value_floor)
        H_mu = torch.clamp(H_mu, min=value_floor)
    sel = torch.as_tensor(np.asarray(chose_newton, dtype=bool))[None, :]
    return torch.where(sel, Hn, H_mu)


def unrolled_loss(V, W, H_init, H0, K, masks, eps=EPS, alpha=ALPHA, value_floor=0.0, perturb=None):
    """L = ||H_K - H0||^2 over K frozen-selection updates, as a torch graph.
    ``perturb``: None, or a function k -> (nA, nB) for update k (see
    h_update_torch)."""
    H = H_init
    for k in range(K):
        H = h_update_torch(V, W, H, masks[k], eps, alpha, value_floor, None if perturb is None else perturb(k))
    return ((H - H0) ** 2).sum(), H


def unrolled_h_grad(V, W, H_init, H0, K, masks=None, eps=EPS, alpha=ALPHA, value_floor=0.0, perturb=None):
    """Loss and gradients (dL/dW, dL/dV, dL/dH_init) of L = ||H_K - H0||^2.

    ``masks`` (K boolean arrays of length T) freeze the selections; by default
    they come from the NumPy oracle's forward pass from the same inputs.
    ``perturb`` as in unrolled_loss (sensitivity probe; default None).
    Returns (L, H_K, dW, dV, dH_init) as float64 NumPy arrays."""
    if masks is None:
        _, masks = unrolled_h(V, W, H_init, K, eps, alpha, value_floor)
    t = lambda x: torch.tensor(np.asarray(x, dtype=np.float64), requires_grad=True)
    Vt, Wt, Ht = t(V), t(W), t(H_init)
    H0t = torch.tensor(np.asarray(H0, dtype=np.float64))
    L, HK = unrolled_loss(Vt, Wt, Ht, H0t, K, masks, eps, alpha, value_floor, perturb)
    L.backward()
    g = lambda x: x.grad.numpy() if x.grad is not None else np.zeros(tuple(x.shape))
    return float(L), HK.detach().numpy(), g(Wt), g(Vt), g(Ht)
