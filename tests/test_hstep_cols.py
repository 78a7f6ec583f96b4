"""The one-kernel H half-step (R <= 64, T >= 4096: a workgroup per 16 columns,
candidates, costs and choice without split partials) against the FP64 oracle,
through the C ABI: its candidates, one half-step from identical states (the
decisions re-scored in FP64 from the kernel's own candidates and compared with
the oracle's), whole iterations, degenerate columns and checked mode.  Shapes
have ragged sub-tiles (N mod 64), ragged column blocks (T mod 16) and every
rank-group count (R in 1..16, 17..32, 33..48, 49..64)."""
import numpy as np
import pytest

import oracle
from paper_1301_3389_amd import synth
from parity_util import (FLOOR32, STEP_TOL, TRAJ_TOL, cost_err, gpu, host, log_result, rel_cols)
from test_parity_fwd import _check_update, _problem

pytestmark = pytest.mark.gpu

SHAPES = [
    # N, T, R, zero_frac, seed
    (300, 4100, 64, 0.1, 21),
    (130, 4096, 37, 0.2, 22),
    (64, 5003, 10, 0.0, 23),
    (257, 4099, 20, 0.05, 24),
    (1, 4096, 3, 0.0, 25),
    (700, 4200, 49, 0.1, 26),
]


@pytest.mark.parametrize("shape", SHAPES)
def test_hcols_candidates(dna, shape):
    V, W, H = _problem(*shape)
    Xmu, Xn = dna.candidates(0, gpu(V), gpu(W), gpu(H))
    r = oracle.h_step(V, W, H, value_floor=FLOOR32)
    e_mu = rel_cols(host(Xmu), r.X_mu, 0).max()
    e_n = rel_cols(host(Xn), r.X_newton, 0).max()
    log_result("hcols_candidates", {"shape": shape, "err_mu": float(e_mu), "err_newton": float(e_n)})
    assert e_mu <= STEP_TOL
    assert e_n <= STEP_TOL


@pytest.mark.parametrize("shape", SHAPES)
def test_hcols_update(dna, shape):
    V, W, H = _problem(*shape)
    _check_update(dna, V, W, H, 0, "hcols_update")


@pytest.mark.parametrize("shape", SHAPES)
def test_hcols_update_regularised(dna, shape):
    """lambda > 0 (eq. 2): c = W^t 1 + lambda in the gain and the rescaling."""
    V, W, H = _problem(*shape)
    Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
    dna.update_H(Vg, Wg, Hg, lam=0.3)
    r = oracle.h_step(V, W, H, value_floor=FLOOR32, lam=0.3)
    assert rel_cols(host(Hg), r.X, 0).max() <= STEP_TOL


def test_hcols_empty_columns(dna):
    """All-zero data columns (including the last, ragged block's) and rows."""
    V, W, H = _problem(200, 4100, 12, 0.1, 27)
    for t in (5, 77, 4096, 4099):
        V[:, t] = 0.0
    V[3, :] = 0.0
    _check_update(dna, V, W, H, 0, "hcols_update_empty")


@pytest.mark.parametrize("shape", [SHAPES[0], SHAPES[2]])
def test_hcols_trajectory(dna, shape):
    """dna_iterate (the one-kernel H step, its row sums handed to the
    normalisation) against the oracle's fit_dna: KL within 1e-4 after each of
    8 iterations and non-increasing."""
    V, W, H = _problem(*shape)
    Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
    kls = host(dna.fit(Vg, Wg, Hg, 8, method="dna", record_kl=True))
    ref = np.array(oracle.fit_dna(V, W, H, 8, value_floor=FLOOR32).kl)
    rel = np.abs(kls - ref) / np.abs(ref)
    log_result("hcols_trajectory", {"shape": shape, "max_rel": float(rel.max())})
    assert rel.max() <= TRAJ_TOL
    assert np.all(np.diff(kls) <= 1e-6 * np.abs(kls[:-1]))


def test_hcols_iterate_matches_separate_calls(dna):
    """dna_iterate against dna_update_H / normalize / dna_update_W / normalize
    called one by one: the same kernels on the same state, so the KL agrees to
    1e-6 after three iterations."""
    V, W, H = _problem(*SHAPES[3])
    Vg = gpu(V)
    Wa, Ha = gpu(W), gpu(H)
    dna.normalize(0, Wa, Ha)
    Wb, Hb = Wa.clone(), Ha.clone()
    dna.iterate(Vg, Wa, Ha, 3)
    for _ in range(3):
        dna.dna_iteration(Vg, Wb, Hb)
    kla, klb = dna.kl_cost(Vg, Wa, Ha).item(), dna.kl_cost(Vg, Wb, Hb).item()
    assert abs(kla - klb) <= 1e-6 * abs(klb)


def test_hcols_deterministic(dna):
    V, W, H = _problem(*SHAPES[0])
    outs = []
    for _ in range(2):
        Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
        dna.iterate(Vg, Wg, Hg, 2)
        outs.append((host(Wg), host(Hg)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_hcols_checked_mode(dna):
    V, W, H = _problem(100, 4096, 8, 0.0, 28)
    Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
    dna.update_H(Vg, Wg, Hg, checked=True)          # valid input passes
    Wbad = W.copy()
    Wbad[:, 2] = 0.0                                # zero column sum
    with pytest.raises(dna.DNAError) as e:
        dna.update_H(Vg, gpu(Wbad), gpu(H), checked=True)
    assert e.value.status == 3
