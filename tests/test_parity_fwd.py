"""GPU parity of the forward path against the FP64 oracle, through the C ABI.

Every comparison starts both sides from the same float32 state (the oracle
upcasts it).  Shapes span several 128-wide tiles with ragged tails, plus the
degenerate cases (R = 1, T = 1, N = 1, all-zero columns / rows)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import dna_oracle as O
from paper_1301_3389_amd import synth
from parity_util import (FLOOR32, SELECT_TIE, STATE_TIE, STEP_TOL, TRAJ_TOL, cost_err, gpu, host, log_result,
                         recon_gap, rel_cols, rescore, selection_report)

pytestmark = pytest.mark.gpu

SHAPES = [
    # N, T, R, zero_frac, seed
    (300, 333, 37, 0.2, 1),
    (257, 130, 10, 0.0, 2),
    (64, 64, 64, 0.3, 3),
    (1000, 515, 64, 0.1, 4),
    (130, 200, 1, 0.0, 5),
    (5, 7, 3, 0.0, 6),
    (130, 1, 4, 0.0, 7),
    (1, 90, 3, 0.0, 8),
    (200, 300, 129, 0.05, 9),
    (150, 170, 100, 0.1, 10),    # 64 < R <= 128: the register-resident candidate forms
    (2600, 150, 80, 0.1, 13),    # many contraction splits over few columns: folded before the candidates
    (2600, 150, 40, 0.1, 14),    # the same through the fused kernels: 41 cost partials per column
    (2100, 2300, 96, 0.1, 15),   # contractions of >= 2048 indices both ways: chunked gradient sums
    (64, 16384, 200, 0.1, 16),   # 128 < R <= 512 over whole rounds of 1024-thread blocks: the H-side
                                 # candidates keep 16 rows per thread in registers (R ragged)
    (300, 4100, 48, 0.1, 17),    # 32 < R <= 64 with T >= 2048: the fused W step's chunked u_c
]


def _problem(N, T, R, zf, seed):
    w = synth.random_problem(N, T, R, seed, zero_frac=zf)
    V = w.V.copy()
    # guarantee every column and row of V has a positive entry unless a test
    # wants empty ones
    V[0, :] = np.maximum(V[0, :], 1.0)
    V[:, 0] = np.maximum(V[:, 0], 1.0)
    return V, w.W, w.H


@pytest.mark.parametrize("shape", SHAPES)
def test_kl_cost(dna, shape):
    V, W, H = _problem(*shape)
    got = dna.kl_cost(gpu(V), gpu(W), gpu(H)).item()
    ref = oracle.kl_cost(V, W, H)
    assert got == pytest.approx(ref, rel=1e-6)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("side", [0, 1])
def test_gradient_hessian(dna, shape, side):
    V, W, H = _problem(*shape)
    A, B = dna.gradient_hessian(side, gpu(V), gpu(W), gpu(H))
    r = (oracle.h_step if side == 0 else oracle.w_step)(V, W, H, value_floor=FLOOR32)
    A, B = host(A), host(B)
    # A = g - 1 with g = u/c the MU gain: compare through g, relative
    errA = np.max(np.abs(A - r.A) / (np.abs(1.0 + r.A) + 1e-30))
    errB = rel_cols(B, r.B, axis=0 if side == 0 else 1).max()
    log_result("gradient_hessian", {"shape": shape, "side": side, "errA": float(errA), "errB": float(errB)})
    assert errA <= STEP_TOL
    assert errB <= STEP_TOL


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("side", [0, 1])
def test_candidates(dna, shape, side):
    V, W, H = _problem(*shape)
    Xmu, Xn = dna.candidates(side, gpu(V), gpu(W), gpu(H))
    r = (oracle.h_step if side == 0 else oracle.w_step)(V, W, H, value_floor=FLOOR32)
    ax = 0 if side == 0 else 1
    e_mu = rel_cols(host(Xmu), r.X_mu, ax).max()
    e_n = rel_cols(host(Xn), r.X_newton, ax).max()
    log_result("candidates", {"shape": shape, "side": side, "err_mu": float(e_mu), "err_newton": float(e_n)})
    assert e_mu <= STEP_TOL
    assert e_n <= STEP_TOL


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("side", [0, 1])
def test_select_from_identical_candidates(dna, shape, side):
    """Steps 7-9, 12-15 given the GPU's own candidates: the oracle re-scores them in
    float64; every decision with a relative margin above 1e-12 must agree."""
    V, W, H = _problem(*shape)
    Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
    Xmu, Xn = dna.candidates(side, Vg, Wg, Hg)
    F = Wg if side == 0 else Hg
    out, m, d, g = dna.select(side, Vg, F, Xmu, Xn)
    xm, xn = host(Xmu), host(Xn)
    if side == 0:
        d_mu = O.partial_cost(V, W.astype(float) @ xm, 0)
        d_n = O.partial_cost(V, W.astype(float) @ xn, 0)
    else:
        d_mu = O.partial_cost(V, xm @ H.astype(float), 1)
        d_n = O.partial_cost(V, xn @ H.astype(float), 1)
    choose = d_n < d_mu
    margin = d_mu - d_n
    if side == 0:
        zgap = recon_gap(W.astype(float) @ xm, W.astype(float) @ xn, 0)
    else:
        zgap = recon_gap(xm @ H.astype(float), xn @ H.astype(float), 1)
    rep = selection_report(host(m), choose, margin, d_mu, SELECT_TIE, zgap)
    d_ref = np.where(choose, d_n, d_mu)
    vsum = V.astype(float).sum(axis=0 if side == 0 else 1)
    agree = host(m).astype(bool) == choose
    err_d = cost_err(host(d)[agree], d_ref[agree], vsum[agree])
    err_m = cost_err(host(g), margin, vsum)
    log_result("select_identical", {"shape": shape, "side": side, **rep, "err_dsel": err_d, "err_margin": err_m})
    assert rep["n_flips_above_tie"] == 0, rep
    assert err_d <= 1.0
    assert err_m <= 1.0
    kept = np.where(host(m).astype(bool)[None, :] if side == 0 else host(m).astype(bool)[:, None], xn, xm)
    assert np.array_equal(host(out), kept)


def _check_update(dna, V, W, H, side, name):
    Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
    # the GPU's own candidates from the same state (the kernels the update runs)
    Xmu, Xn = dna.candidates(side, Vg, Wg, Hg)
    if side == 0:
        m, d, g = dna.update_H(Vg, Wg, Hg, mask=True, d_sel=True, margin=True)
        got = host(Hg)
        r = oracle.h_step(V, W, H, value_floor=FLOOR32)
    else:
        m, d, g = dna.update_W(Vg, Wg, Hg, mask=True, d_sel=True, margin=True)
        got = host(Wg)
        r = oracle.w_step(V, W, H, value_floor=FLOOR32)
    ax = 0 if side == 0 else 1
    mask = host(m).astype(bool)
    Wd, Hd = W.astype(float), H.astype(float)
    zgap = recon_gap(Wd @ r.X_mu, Wd @ r.X_newton, 0) if side == 0 else recon_gap(r.X_mu @ Hd, r.X_newton @ Hd, 1)
    rep = selection_report(mask, r.chose_newton, r.margin, r.d_mu, STATE_TIE, zgap)
    ch, mg, dm, zg = rescore(V, W if side == 0 else H, host(Xmu), host(Xn), side)
    rep_own = selection_report(mask, ch, mg, dm, SELECT_TIE, zg)
    same = mask == r.chose_newton
    err = rel_cols(got, r.X, ax)[same]
    vsum = V.astype(float).sum(axis=0 if side == 0 else 1)
    # where the selections differ the GPU result must equal the oracle's other candidate
    sel = r.chose_newton[None, :] if side == 0 else r.chose_newton[:, None]
    other = np.where(sel, r.X_mu, r.X_newton)
    err_other = rel_cols(got, other, ax)[~same]
    err_d = cost_err(host(d)[same], r.d_sel[same], vsum[same])
    log_result(name, {"side": side, **rep, "max_err": float(err.max()) if err.size else 0.0,
                      "err_dsel": err_d, "own": rep_own})
    assert rep_own["n_flips_above_tie"] == 0, rep_own
    assert rep["n_flips_above_tie"] == 0, rep
    assert err.size == 0 or err.max() <= STEP_TOL
    assert err_other.size == 0 or err_other.max() <= STEP_TOL
    assert err_d <= 1.0


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("side", [0, 1])
def test_update_from_identical_state(dna, shape, side):
    V, W, H = _problem(*shape)
    _check_update(dna, V, W, H, side, "update")


@pytest.mark.parametrize("shape", SHAPES[:4])
@pytest.mark.parametrize("side", [0, 1])
@pytest.mark.parametrize("with_cost", [False, True])
def test_mu_update(dna, shape, side, with_cost):
    V, W, H = _problem(*shape)
    Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
    d = dna.mu_update(side, Vg, Wg, Hg, with_cost=with_cost)
    if side == 0:
        ref, dref = oracle.mu_h_step(V, W, H, value_floor=FLOOR32)
        err = rel_cols(host(Hg), ref, 0).max()
    else:
        ref, dref = oracle.mu_w_step(V, W, H, value_floor=FLOOR32)
        err = rel_cols(host(Wg), ref, 1).max()
    assert err <= STEP_TOL
    if with_cost:
        np.testing.assert_allclose(host(d), dref, rtol=STEP_TOL)


@pytest.mark.parametrize("shape", SHAPES[:4])
@pytest.mark.parametrize("side", [0, 1])
def test_normalize(dna, shape, side):
    V, W, H = _problem(*shape)
    Wg, Hg = gpu(W), gpu(H)
    dna.normalize(side, Wg, Hg)
    if side == 0:
        Wr, Hr = oracle.normalize_w_columns(W, H)
    else:
        Wr, Hr = oracle.normalize_h_rows(W, H)
    np.testing.assert_allclose(host(Wg), Wr, rtol=2e-7)
    np.testing.assert_allclose(host(Hg), Hr, rtol=2e-7)


def test_empty_columns_and_rows(dna):
    """All-zero data columns / rows: s_t = 0 sends both candidates to 0 (tie -> MU)."""
    V, W, H = _problem(150, 140, 6, 0.1, 11)
    V[:, 5] = 0.0
    V[:, 77] = 0.0
    V[3, :] = 0.0
    V[140, :] = 0.0
    for side in (0, 1):
        _check_update(dna, V, W, H, side, "update_empty")


def test_planted_fixed_point(dna):
    rng = np.random.default_rng(12)
    W0 = rng.uniform(0.2, 1.0, (140, 5)).astype(np.float32)
    H0 = rng.uniform(0.2, 1.0, (5, 150)).astype(np.float32)
    V = (W0.astype(float) @ H0.astype(float)).astype(np.float32)
    Vg, Wg, Hg = gpu(V), gpu(W0), gpu(H0)
    dna.update_H(Vg, Wg, Hg)
    assert rel_cols(host(Hg), H0, 0).max() <= 1e-5
    dna.update_W(Vg, Wg, Hg)
    assert rel_cols(host(Wg), W0, 1).max() <= 1e-5


def test_checked_mode_domain_errors(dna):
    V, W, H = _problem(64, 64, 4, 0.0, 13)
    Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
    dna.update_H(Vg, Wg, Hg, checked=True)          # valid input passes
    Wbad = W.copy()
    Wbad[:, 2] = 0.0                                # zero column sum
    with pytest.raises(dna.DNAError) as e:
        dna.update_H(Vg, gpu(Wbad), gpu(H), checked=True)
    assert e.value.status == 3
    Vbad = V.copy()
    Vbad[3, 3] = np.nan
    with pytest.raises(dna.DNAError) as e:
        dna.kl_cost(gpu(Vbad), Wg, Hg, checked=True)
    assert e.value.status == 4
    Hneg = H.copy()
    Hneg[1, 1] = -1.0
    with pytest.raises(dna.DNAError) as e:
        dna.update_W(Vg, Wg, gpu(Hneg), checked=True)
    assert e.value.status == 3


def test_deterministic(dna):
    """Fixed-order reductions: two runs give bit-identical results."""
    V, W, H = _problem(1000, 515, 64, 0.1, 4)
    outs = []
    for _ in range(2):
        Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
        dna.dna_iteration(Vg, Wg, Hg)
        outs.append((host(Wg), host(Hg)))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert np.array_equal(outs[0][1], outs[1][1])


# (1000, 4100, 37): the one-kernel H step and normalisations over more than 128
# parts with R not a multiple of the 16-column W tiles; (1024, 10240, 512): the
# W-step normalisation over 256 parts at R = 512 takes longer H chunks (two of
# 4096 entries and a last one of 2048)
@pytest.mark.parametrize("shape", [SHAPES[0], SHAPES[3], SHAPES[6], SHAPES[7], (1024, 2300, 64, 0.1, 11),
                                   (200, 2100, 100, 0.0, 12), (1000, 4100, 37, 0.1, 18),
                                   (1024, 10240, 512, 0.1, 19)])
def test_iterate_matches_separate_calls(dna, shape):
    """dna_iterate (sums handed from each normalisation to the next half-step)
    against the four separate entry points, from the same state: the state after
    one and after three iterations agrees to float32 rounding except where a
    selection tie flipped, and the KL agrees to 1e-6."""
    V, W, H = _problem(*shape)
    Vg = gpu(V)
    Wa, Ha = gpu(W), gpu(H)
    dna.normalize(0, Wa, Ha)
    Wb, Hb = Wa.clone(), Ha.clone()
    for k in (1, 2):
        dna.iterate(Vg, Wa, Ha, k)
        for _ in range(k):
            dna.dna_iteration(Vg, Wb, Hb)
        kla, klb = dna.kl_cost(Vg, Wa, Ha).item(), dna.kl_cost(Vg, Wb, Hb).item()
        assert abs(kla - klb) <= 1e-6 * abs(klb)
        for a, b in ((Wa, Wb), (Ha, Hb)):
            a, b = host(a), host(b)
            rel = np.abs(a - b) / np.maximum(np.abs(b), 1e-30)
            assert np.mean(rel > 1e-4) <= 0.01, (k, float(rel.max()))
    Wz, Hz = Wa.clone(), Ha.clone()
    dna.iterate(Vg, Wz, Hz, 0)
    assert torch.equal(Wz, Wa) and torch.equal(Hz, Ha)


@pytest.mark.parametrize("with_cost", [False, True])
def test_mu_iterate_matches_separate_calls(dna, with_cost):
    """mu_iterate runs the same kernels as mu_update / dna_normalize in the same
    order: the state after three iterations is bit-identical."""
    V, W, H = _problem(*SHAPES[0])
    Vg = gpu(V)
    Wa, Ha = gpu(W), gpu(H)
    dna.normalize(0, Wa, Ha)
    Wb, Hb = Wa.clone(), Ha.clone()
    dna.mu_iterate(Vg, Wa, Ha, 3, with_cost=with_cost)
    for _ in range(3):
        dna.mu_update(0, Vg, Wb, Hb, with_cost=with_cost)
        dna.normalize(1, Wb, Hb)
        dna.mu_update(1, Vg, Wb, Hb, with_cost=with_cost)
        dna.normalize(0, Wb, Hb)
    assert torch.equal(Wa, Wb) and torch.equal(Ha, Hb)


def _trajectory(dna, V, W, H, iters, method):
    Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
    kls = host(dna.fit(Vg, Wg, Hg, iters, method=method, record_kl=True))
    ref = (oracle.fit_dna if method == "dna" else oracle.fit_mu)(V, W, H, iters, value_floor=FLOOR32)
    rel = np.abs(kls - np.array(ref.kl)) / np.abs(np.array(ref.kl))
    return kls, np.array(ref.kl), rel


@pytest.mark.parametrize("method", ["dna", "mu"])
def test_trajectory_config1(dna, method):
    """Workload 1 (200 x 300, R = 10): 20 alternating iterations, KL within 1e-4."""
    w = synth.config1()
    kls, ref, rel = _trajectory(dna, w.V, w.W, w.H, 20, method)
    log_result("trajectory_config1", {"method": method, "max_rel": float(rel.max()),
                                      "kl_last": float(kls[-1]), "kl_ref_last": float(ref[-1])})
    assert rel.max() <= TRAJ_TOL
    assert np.all(np.diff(kls) <= 1e-6 * np.abs(kls[:-1]))    # non-increasing (Sec. 2.4)


@pytest.mark.parametrize("method", ["dna", "mu"])
def test_trajectory_config2_slab(dna, method):
    """A 1024 x 1024 slab of the workload-2 recipe (R = 64), 30 iterations."""
    w = synth.config2()
    V, W, H = w.V[:, :1024].copy(), w.W, w.H[:, :1024].copy()
    kls, ref, rel = _trajectory(dna, V, W, H, 30, method)
    log_result("trajectory_config2_slab", {"method": method, "max_rel": float(rel.max())})
    assert rel.max() <= TRAJ_TOL


def test_trajectory_config2_long(dna):
    """The workload-2 iteration count (200 DNA iterations) on a 1024 x 512 slab:
    long enough for many entries to shrink towards the float32 range limit, which
    the value floor must keep on the oracle's trajectory."""
    w = synth.config2()
    V, W, H = w.V[:, :512].copy(), w.W, w.H[:, :512].copy()
    kls, ref, rel = _trajectory(dna, V, W, H, 200, "dna")
    log_result("trajectory_config2_long", {"max_rel": float(rel.max()), "kl_last": float(kls[-1]),
                                           "kl_ref_last": float(ref[-1])})
    assert rel.max() <= TRAJ_TOL


def _golden_config2():
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config2_trajectory.json")
    with open(path) as f:
        return json.load(f)


def test_trajectory_config2_full(dna):
    """The full N=1024 T=8192 R=64 workload, 200 DNA iterations in the launch
    configuration the benchmark times (one dna_iterate call per iteration),
    against the FP64 oracle's trajectory with the float32 value floor
    (tests/golden/config2_trajectory.json, written by the committed script that
    calls only the oracle): relative KL within 1e-4 after every iteration."""
    w = synth.config2()
    ref = np.array(_golden_config2()["dna_floor"])
    Vg, Wg, Hg = gpu(w.V), gpu(w.W), gpu(w.H)
    kls = host(dna.fit(Vg, Wg, Hg, 200, method="dna", record_kl=True))
    rel = np.abs(kls - ref) / np.abs(ref)
    log_result("trajectory_config2_full", {"max_rel": float(rel.max()), "kl_last": float(kls[-1]),
                                           "kl_ref_last": float(ref[-1])})
    assert rel.max() <= TRAJ_TOL


def test_mu_target_kl_config2_full(dna):
    """The benchmark's target KL (float32 GPU MU, 1000 iterations from the same
    start on the full N=1024 T=8192 R=64 workload) against the FP64 oracle's
    1000-iteration MU trajectory: within 1e-4 at every 50th iteration and at the
    end."""
    ref = np.array(_golden_config2()["mu_floor"])
    w = synth.config2()
    Vg, Wg, Hg = gpu(w.V), gpu(w.W), gpu(w.H)
    dna.normalize(0, Wg, Hg)
    got = [dna.kl_cost(Vg, Wg, Hg).item()]
    for k in range(20):
        dna.mu_iterate(Vg, Wg, Hg, 50)
        got.append(dna.kl_cost(Vg, Wg, Hg).item())
    got = np.array(got)
    rel = np.abs(got - ref[::50]) / ref[::50]
    log_result("mu_target_kl_config2_full", {"max_rel": float(rel.max()), "kl_gpu": float(got[-1]),
                                             "kl_oracle": float(ref[-1])})
    assert rel.max() <= TRAJ_TOL


# --------------------------------------------------------------------------- full sizes, sampled

def _sampled_step(dna, V, W, H, n_cols=24, n_rows=24, seed=0):
    """One H step and one W step at full size on the GPU, checked on sampled columns
    (H step: columns are independent) and sampled rows (W step: rows independent)."""
    rng = np.random.default_rng(seed)
    N, T = V.shape
    Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
    cols = np.sort(rng.choice(T, size=min(n_cols, T), replace=False))
    rows = np.sort(rng.choice(N, size=min(n_rows, N), replace=False))
    H1 = Hg.clone()
    Xmu, Xn = dna.candidates(0, Vg, Wg, Hg)
    m, d, g = dna.update_H(Vg, Wg, H1, mask=True, d_sel=True, margin=True)
    r = oracle.h_step(V[:, cols], W, H[:, cols], value_floor=FLOOR32)
    ch, mg, dm, zo = rescore(V[:, cols], W, host(Xmu)[:, cols], host(Xn)[:, cols], 0)
    del Xmu, Xn
    got = host(H1)[:, cols]
    mask = host(m)[cols].astype(bool)
    Wd = W.astype(float)
    zg = recon_gap(Wd @ r.X_mu, Wd @ r.X_newton, 0)
    rep_h = selection_report(mask, r.chose_newton, r.margin, r.d_mu, STATE_TIE, zg)
    rep_h["own"] = selection_report(mask, ch, mg, dm, SELECT_TIE, zo)
    same = mask == r.chose_newton
    err_h = rel_cols(got, r.X, 0)[same]
    W1 = Wg.clone()
    Xmu, Xn = dna.candidates(1, Vg, Wg, Hg)
    m2, d2, g2 = dna.update_W(Vg, W1, Hg, mask=True, d_sel=True, margin=True)
    rw = oracle.w_step(V[rows], W[rows], H, value_floor=FLOOR32)
    ch, mg, dm, zo = rescore(V[rows], H, host(Xmu)[rows], host(Xn)[rows], 1)
    del Xmu, Xn
    gotw = host(W1)[rows]
    maskw = host(m2)[rows].astype(bool)
    Hd = H.astype(float)
    zgw = recon_gap(rw.X_mu @ Hd, rw.X_newton @ Hd, 1)
    rep_w = selection_report(maskw, rw.chose_newton, rw.margin, rw.d_mu, STATE_TIE, zgw)
    rep_w["own"] = selection_report(maskw, ch, mg, dm, SELECT_TIE, zo)
    samew = maskw == rw.chose_newton
    err_w = rel_cols(gotw, rw.X, 1)[samew]
    return rep_h, err_h, rep_w, err_w


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_full_size_sampled(dna, k):
    w = synth.config(k)
    rep_h, err_h, rep_w, err_w = _sampled_step(dna, w.V, w.W, w.H, seed=k)
    log_result("full_size_sampled", {"config": k, "h": rep_h, "w": rep_w,
                                     "err_h": float(err_h.max()) if err_h.size else 0.0,
                                     "err_w": float(err_w.max()) if err_w.size else 0.0,
                                     "meta": {kk: v for kk, v in w.meta.items() if isinstance(v, (int, float))}})
    assert rep_h["n_flips_above_tie"] == 0 and rep_w["n_flips_above_tie"] == 0
    assert rep_h["own"]["n_flips_above_tie"] == 0 and rep_w["own"]["n_flips_above_tie"] == 0
    assert err_h.size == 0 or err_h.max() <= STEP_TOL
    assert err_w.size == 0 or err_w.max() <= STEP_TOL
    del w
    torch.cuda.empty_cache()


def test_concurrent_streams_match_sequential(dna):
    """Independent problems issued on three streams at once, their iterations
    interleaved (each stream gets its own workspace from the binding), end
    bit-identical to the same problems run one after another."""
    probs = [_problem(300, 333, 37, 0.2, s) for s in (21, 22, 23)]
    seq = []
    for V, W, H in probs:
        Vg, Wg, Hg = gpu(V), gpu(W), gpu(H)
        dna.normalize(0, Wg, Hg)
        for _ in range(4):
            dna.iterate(Vg, Wg, Hg, 1)
        seq.append((host(Wg), host(Hg)))
    state = [(gpu(V), gpu(W), gpu(H)) for V, W, H in probs]
    streams = [torch.cuda.Stream() for _ in probs]
    for st, (Vg, Wg, Hg) in zip(streams, state):
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            dna.normalize(0, Wg, Hg)
    for _ in range(4):
        for st, (Vg, Wg, Hg) in zip(streams, state):
            with torch.cuda.stream(st):
                dna.iterate(Vg, Wg, Hg, 1)
    torch.cuda.synchronize()
    for (Wr, Hr), (_, Wg, Hg) in zip(seq, state):
        assert np.array_equal(host(Wg), Wr) and np.array_equal(host(Hg), Hr)
