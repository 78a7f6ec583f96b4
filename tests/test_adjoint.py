"""Adjoint of K unrolled DNA H-updates (W fixed), loss ||H_K - H0||^2.

CPU: the oracle's reference gradient (torch float64 autograd with frozen
selections) is pinned to central finite differences of the NumPy oracle's own
forward pass, entry by entry, away from branch boundaries.
GPU: the hand-written HIP adjoint (through the C ABI, behind
torch.autograd.Function) against the oracle gradient with the GPU's selections."""
import numpy as np
import pytest
import torch

import oracle
from oracle import adjoint as OA
from oracle import dna_oracle as O
from paper_1301_3389_amd import synth


def _small(seed=0, N=16, R=4, T=8):
    rng = np.random.default_rng(seed)
    W = rng.gamma(0.5, 1.0, (N, R)) + 0.05
    H0 = rng.gamma(0.5, 1.0, (R, T))
    V = rng.poisson(W @ H0 * 3.0).astype(float) + 0.5      # strictly positive data
    H_init = rng.uniform(0.1, 1.0, (R, T))
    return V, W, H_init, H0


def _signature(V, W, H, K):
    """Selections and inner branch states of every update (for kink detection)."""
    sig = []
    for _ in range(K):
        r = oracle.h_step(V, W, H)
        xb = H * r.B
        with np.errstate(divide="ignore", invalid="ignore"):
            gain = np.where(r.A < 0, xb / (xb - r.A), 0.0)
            step = np.where(r.B > 0, r.A / np.where(r.B > 0, r.B, 1.0), np.inf)
        sig.append(np.concatenate([r.chose_newton.ravel(), (r.A < 0).ravel(),
                                   ((r.A < 0) & (gain < oracle.EPS)).ravel(),
                                   ((r.A >= 0) & (step > oracle.ALPHA * H)).ravel()]))
        H = r.X
    return np.concatenate(sig), H


def _loss(V, W, H_init, H0, K):
    Hs, _ = oracle.unrolled_h(V, W, H_init, K)
    return float(((Hs[-1] - H0) ** 2).sum())


def test_torch_transcription_matches_numpy_oracle():
    V, W, H, H0 = _small(1)
    Hs, masks = oracle.unrolled_h(V, W, H, 4)
    t = lambda x: torch.tensor(x, dtype=torch.float64)
    Ht = t(H)
    for k in range(4):
        Ht = OA.h_update_torch(t(V), t(W), Ht, masks[k])
        np.testing.assert_allclose(Ht.numpy(), Hs[k + 1], rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_reference_gradient_matches_finite_differences(seed):
    """Central differences of the NumPy forward (step 1e-6 relative) against the
    autograd reference gradient, for every entry of W, V and H_init whose
    perturbation leaves all selections and branches unchanged."""
    K = 3
    V, W, H, H0 = _small(seed)
    L, HK, dW, dV, dH = OA.unrolled_h_grad(V, W, H, H0, K)
    base_sig, _ = _signature(V, W, H, K)
    checked = skipped = 0
    worst = 0.0
    for name, X, G in (("W", W, dW), ("V", V, dV), ("H", H, dH)):
        for idx in np.ndindex(X.shape):
            h = 1e-6 * abs(X[idx])
            Xp, Xm = X.copy(), X.copy()
            Xp[idx] += h
            Xm[idx] -= h
            args_p = {"W": (V, Xp, H), "V": (Xp, W, H), "H": (V, W, Xp)}[name]
            args_m = {"W": (V, Xm, H), "V": (Xm, W, H), "H": (V, W, Xm)}[name]
            sp, _ = _signature(*args_p, K)
            sm, _ = _signature(*args_m, K)
            if not (np.array_equal(sp, base_sig) and np.array_equal(sm, base_sig)):
                skipped += 1
                continue
            fd = (_loss(*args_p, H0, K) - _loss(*args_m, H0, K)) / (2 * h)
            scale = max(abs(G[idx]), 1e-3 * np.max(np.abs(G)))
            worst = max(worst, abs(fd - G[idx]) / scale)
            checked += 1
    assert checked > 0.9 * (W.size + V.size + H.size), (checked, skipped)
    assert worst < 1e-5, worst


def test_reference_gradient_k0_is_identity():
    V, W, H, H0 = _small(3)
    L, HK, dW, dV, dH = OA.unrolled_h_grad(V, W, H, H0, 0)
    np.testing.assert_allclose(dH, 2 * (H - H0))
    assert np.all(dW == 0) and np.all(dV == 0)


# --------------------------------------------------------------------------- GPU


def _rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def _gpu_vs_oracle(dna, V, W, H, H0, K):
    cuda = lambda x: torch.tensor(np.asarray(x, dtype=np.float32), device="cuda")
    Wg = cuda(W).requires_grad_(True)
    Vg = cuda(V).requires_grad_(True)
    Hg = cuda(H).requires_grad_(True)
    H0g = cuda(H0)
    HK = dna.unrolled_h(Wg, Vg, Hg, K)
    loss = ((HK - H0g) ** 2).sum()
    loss.backward()
    # the oracle follows the GPU's selections, from the same float32 inputs
    H_ckpt, sel = dna.unrolled_forward(cuda(V), cuda(W), cuda(H), K)
    masks = [m.astype(bool) for m in sel.cpu().numpy()]
    f32 = lambda x: np.asarray(x, dtype=np.float32).astype(np.float64)
    L, HKr, dW, dV, dH = OA.unrolled_h_grad(f32(V), f32(W), f32(H), f32(H0), K, masks=masks,
                                            value_floor=float(np.finfo(np.float32).tiny))
    return {
        "HK": _rel_l2(HK.detach().cpu().numpy(), HKr),
        "dW": _rel_l2(Wg.grad.cpu().numpy(), dW),
        "dV": _rel_l2(Vg.grad.cpu().numpy(), dV),
        "dH": _rel_l2(Hg.grad.cpu().numpy(), dH),
        "loss": abs(loss.item() - L) / L,
        "newton_frac": float(np.mean(masks)) if masks else 0.0,
    }


@pytest.mark.gpu
@pytest.mark.parametrize("seed", [0, 1])
def test_gpu_adjoint_small(dna, seed):
    V, W, H, H0 = _small(seed)
    e = _gpu_vs_oracle(dna, V, W, H, H0, 3)
    from parity_util import log_result
    log_result("adjoint_small", {"seed": seed, **e})
    assert e["HK"] < 1e-5 and e["loss"] < 1e-5
    for k in ("dW", "dV", "dH"):
        assert e[k] < 1e-4, e


@pytest.mark.gpu
def test_gpu_adjoint_medium(dna):
    w = synth.random_problem(150, 300, 20, 21, positive=True)
    rng = np.random.default_rng(5)
    H0 = rng.gamma(0.5, 1.0, (20, 300))
    e = _gpu_vs_oracle(dna, w.V, w.W, w.H, H0, 5)
    from parity_util import log_result
    log_result("adjoint_medium", e)
    assert e["HK"] < 1e-4
    for k in ("dW", "dV", "dH"):
        assert e[k] < 1e-3, e


@pytest.mark.gpu
def test_gpu_adjoint_workload5_columns(dna):
    """The unrolled workload at its real N = 513 and R = 1024 with K = 20, on a
    256-column batch (columns are independent given W, so this is the same
    computation per column; the oracle gradient is exact for the batch)."""
    w = synth.config5(T=256)
    e = _gpu_vs_oracle(dna, w.V, w.W, w.H, w.H0, 20)
    from parity_util import log_result
    log_result("adjoint_workload5_cols", e)
    assert e["HK"] < 1e-3
    for k in ("dW", "dV", "dH"):
        assert e[k] < 1e-2, e


@pytest.mark.gpu
def test_gpu_adjoint_k0(dna):
    V, W, H, H0 = _small(4)
    cuda = lambda x: torch.tensor(np.asarray(x, dtype=np.float32), device="cuda")
    H_ckpt, sel = dna.unrolled_forward(cuda(V), cuda(W), cuda(H), 0)
    g = cuda(2 * (H - H0))
    dW, dV, dH = dna.unrolled_backward(cuda(V), cuda(W), H_ckpt, sel, 0, g)
    assert torch.all(dW == 0) and torch.all(dV == 0)
    assert torch.equal(dH, g)
