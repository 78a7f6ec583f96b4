"""dna_iterate_noalloc (the entry point for callers that cannot allocate) against
dna_iterate with a torch-allocated workspace: same inputs, same kernels, so the
results must be identical, on two calls in a row whose second problem is
smaller than the first (the scratch array keeps the first call's contents)."""
import numpy as np
import pytest
import torch

from paper_1301_3389_amd import synth

pytestmark = pytest.mark.gpu

# (N, T, R, gemm, iters): fused fp32 path, tiled fp32 path (R > 64), the BF16
# form, each followed by a smaller problem
CASES = [
    ((600, 1100, 48, "fp32", 3), (200, 150, 10, "fp32", 2)),
    ((384, 700, 96, "fp32", 2), (130, 70, 70, "fp32", 2)),
    ((512, 640, 80, "bf16", 2), (100, 90, 7, "bf16", 2)),
]


def _state(N, T, R, seed):
    p = synth.random_problem(N, T, R, seed=seed, zero_frac=0.15)
    return [torch.from_numpy(np.ascontiguousarray(x)).cuda() for x in (p.V, p.W, p.H)]


@pytest.mark.parametrize("pair", CASES, ids=lambda c: f"{c[0][:4]}_then_{c[1][:4]}")
def test_noalloc_matches_workspace_call(dna, pair):
    for k, (N, T, R, gemm, iters) in enumerate(pair):
        print(f"noalloc case N={N} T={T} R={R} {gemm} iters={iters} call {k}", flush=True)
        V, W, H = _state(N, T, R, seed=11 + 7 * k + R)
        W1, H1 = W.clone(), H.clone()
        W2, H2 = W.clone(), H.clone()
        dna.iterate(V, W1, H1, iters, gemm=gemm)
        dna.iterate_noalloc(V, W2, H2, iters, gemm=gemm)
        torch.cuda.synchronize()
        assert torch.isfinite(W2).all() and torch.isfinite(H2).all()
        assert torch.equal(W1, W2), (W1 - W2).abs().max().item()
        assert torch.equal(H1, H2), (H1 - H2).abs().max().item()
        # and the call really iterated
        assert not torch.equal(H2, H)


def test_noalloc_rejects_oversized(dna):
    V, W, H = _state(64, 64, 4, seed=3)
    with pytest.raises(dna.DNAError, match="scratch"):
        # claim a large shape: the host check refuses it before any launch
        dna._check(dna._lib_iterate_noalloc(dna._ptr(V), dna._ptr(W), dna._ptr(H), 4096, 32768, 512, 1,
                                            __import__("ctypes").byref(dna.make_opts()), dna._stream()))
