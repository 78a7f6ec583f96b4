"""Seeded synthetic NMF workloads (inputs only, none of the method's arithmetic).

Every generator draws from ``numpy.random.default_rng(seed)`` in float64 and
returns float32 arrays, because the float32 arrays are the state that both the
GPU path and the FP64 oracle start from (the oracle upcasts them).

Shapes and value distributions stand in for the paper's datasets (Sec. 4: dense
face images, sparse term counts, and the speech spectrograms named in Sec. 1),
which are not available:

* ``config(1)``  200 x 300,   R=10   uniform factors, Poisson counts at mean 50
* ``config(2)``  1024 x 8192, R=64   Gamma(0.5) factors, 30%-dense H0, mean 5
* ``config(3)``  4096 x 32768, R=512 spectrogram-like smooth bumps, mean 2
* ``config(4)``  16384 x 20000, R=256 Dirichlet(0.05) columns, ~95% zeros
* ``config(5)``  513 x 4096,  R=1024 fixed W for the unrolled H-solve

Gamma(k, theta) is shape k and scale theta throughout.  The data seed of config
k is 1300+k and the initial-guess seed is 2300+k.
"""
from __future__ import annotations

import dataclasses

import numpy as np

DATA_SEED_BASE = 1300
INIT_SEED_BASE = 2300

SHAPES = {
    1: (200, 300, 10),
    2: (1024, 8192, 64),
    3: (4096, 32768, 512),
    4: (16384, 20000, 256),
    5: (513, 4096, 1024),
}


@dataclasses.dataclass
class Workload:
    """One synthetic problem: data V (N x T), initial guess W (N x R), H (R x T).

    ``W0``/``H0`` are the planted factors V was drawn from (``None`` where not
    kept), ``meta`` records the recipe parameters actually used.
    """
    V: np.ndarray
    W: np.ndarray
    H: np.ndarray
    W0: np.ndarray | None
    H0: np.ndarray | None
    meta: dict


def _poisson_of_product(rng, W0, H0, scale, col_chunk=4096):
    """V = Poisson(scale * W0 @ H0), generated in column chunks to bound memory."""
    N, T = W0.shape[0], H0.shape[1]
    V = np.empty((N, T), dtype=np.float32)
    for t0 in range(0, T, col_chunk):
        t1 = min(T, t0 + col_chunk)
        lam = scale * (W0 @ H0[:, t0:t1])
        V[:, t0:t1] = rng.poisson(lam).astype(np.float32)
    return V


def _product_mean(W0, H0):
    """mean(W0 @ H0) without forming the product: (1^t W0)(H0 1) / (N T)."""
    N, T = W0.shape[0], H0.shape[1]
    return float(W0.sum(axis=0) @ H0.sum(axis=1)) / (N * T)


def uniform_init(N, T, R, seed, lo=0.1, hi=1.0):
    """Initial guess W, H ~ Uniform(lo, hi), float32."""
    rng = np.random.default_rng(seed)
    W = rng.uniform(lo, hi, size=(N, R)).astype(np.float32)
    H = rng.uniform(lo, hi, size=(R, T)).astype(np.float32)
    return W, H


def random_problem(N, T, R, seed, zero_frac=0.0, mean=5.0, positive=False):
    """Generic small problem for parity tests at arbitrary (ragged) shapes.

    W0 ~ Gamma(0.5,1), H0 ~ Gamma(0.5,1), V = Poisson(mean * W0H0/mean(W0H0));
    a further fraction ``zero_frac`` of V entries is zeroed at random.  With
    ``positive`` every entry of V is at least 1e-3 (no zeros at all).
    """
    rng = np.random.default_rng(seed)
    W0 = rng.gamma(0.5, 1.0, size=(N, R))
    H0 = rng.gamma(0.5, 1.0, size=(R, T))
    m = _product_mean(W0, H0)
    V = rng.poisson(mean * (W0 @ H0) / m).astype(np.float32)
    if zero_frac > 0:
        V[rng.random(size=V.shape) < zero_frac] = 0.0
    if positive:
        V = V + np.float32(1e-3)
    W = rng.uniform(0.1, 1.0, size=(N, R)).astype(np.float32)
    H = rng.uniform(0.1, 1.0, size=(R, T)).astype(np.float32)
    return Workload(V, W, H, W0, H0, {"kind": "random", "seed": seed})


def config1():
    N, T, R = SHAPES[1]
    rng = np.random.default_rng(DATA_SEED_BASE + 1)
    W0 = rng.uniform(0.0, 1.0, size=(N, R))
    H0 = rng.uniform(0.0, 1.0, size=(R, T))
    lam = W0 @ H0
    V = (rng.poisson(50.0 * lam / lam.mean()) + 1e-9).astype(np.float32)
    W, H = uniform_init(N, T, R, INIT_SEED_BASE + 1)
    return Workload(V, W, H, W0, H0, {"config": 1, "scale": 50.0})


def config2():
    N, T, R = SHAPES[2]
    rng = np.random.default_rng(DATA_SEED_BASE + 2)
    W0 = rng.gamma(0.5, 1.0, size=(N, R))
    H0 = rng.gamma(0.5, 1.0, size=(R, T)) * (rng.random(size=(R, T)) < 0.3)
    scale = 5.0 / _product_mean(W0, H0)
    V = _poisson_of_product(rng, W0, H0, scale)
    W, H = uniform_init(N, T, R, INIT_SEED_BASE + 2)
    return Workload(V, W, H, W0, H0, {"config": 2, "scale": scale})


def spectrogram_bases(rng, N, R):
    """Smooth Gamma-pdf bumps over the row index, unit column sums.

    Column r has shape k_r ~ U(2,8), mode m_r ~ U(0.02N, 0.9N) and scale
    m_r/(k_r-1), so its maximum sits at row m_r.
    """
    n = np.arange(1, N + 1, dtype=np.float64)[:, None]
    k = rng.uniform(2.0, 8.0, size=R)[None, :]
    mode = rng.uniform(0.02 * N, 0.9 * N, size=R)[None, :]
    theta = mode / (k - 1.0)
    logpdf = (k - 1.0) * np.log(n / theta) - n / theta
    logpdf -= logpdf.max(axis=0, keepdims=True)
    W0 = np.exp(logpdf)
    return W0 / W0.sum(axis=0, keepdims=True)


def config3(T=None):
    N, T_full, R = SHAPES[3]
    T = T_full if T is None else T
    rng = np.random.default_rng(DATA_SEED_BASE + 3)
    W0 = spectrogram_bases(rng, N, R)
    H0 = rng.gamma(0.3, 1.0, size=(R, T_full))[:, :T]
    scale = 2.0 / _product_mean(W0, H0)
    V = _poisson_of_product(rng, W0, H0, scale)
    W, H = uniform_init(N, T_full, R, INIT_SEED_BASE + 3)
    return Workload(V, W, H[:, :T], W0, H0, {"config": 3, "scale": scale})


def calibrate_count_scale(W0, H0, target_zero_frac=0.95, sample_cols=512):
    """kappa such that mean(exp(-kappa * W0 H0)) = target on a column sample.

    exp(-lambda) is the Poisson probability of a zero, so this fixes the
    expected fraction of zero counts.  Bisection in log(kappa).
    """
    Hs = H0[:, :sample_cols]
    lam = W0 @ Hs
    lo, hi = -20.0, 10.0
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        z = float(np.exp(-np.exp(mid) * lam).mean())
        if z > target_zero_frac:
            lo = mid
        else:
            hi = mid
    return float(np.exp(0.5 * (lo + hi)))


def config4(T=None, target_zero_frac=0.95):
    N, T_full, R = SHAPES[4]
    T = T_full if T is None else T
    rng = np.random.default_rng(DATA_SEED_BASE + 4)
    G = rng.gamma(0.05, 1.0, size=(N, R))
    W0 = G / np.maximum(G.sum(axis=0, keepdims=True), 1e-300)
    H0 = rng.gamma(1.0, 20.0, size=(R, T_full))
    kappa = calibrate_count_scale(W0, H0, target_zero_frac)
    H0 = H0[:, :T]
    V = _poisson_of_product(rng, W0, H0, kappa)
    W, H = uniform_init(N, T_full, R, INIT_SEED_BASE + 4)
    zero_frac = float((V == 0).mean())
    return Workload(V, W, H[:, :T], W0, H0,
                    {"config": 4, "kappa": kappa, "zero_frac": zero_frac})


def config5(T=None):
    """Fixed W (513 x 1024), planted H0 and V = Poisson(W H0); H_init ~ U(0.1,1)."""
    N, T_full, R = SHAPES[5]
    T = T_full if T is None else T
    rng = np.random.default_rng(DATA_SEED_BASE + 5)
    W = rng.gamma(0.5, 1.0, size=(N, R))
    H0 = rng.gamma(0.5, 1.0, size=(R, T_full))[:, :T]
    V = _poisson_of_product(rng, W, H0, 1.0)
    init = np.random.default_rng(INIT_SEED_BASE + 5)
    H_init = init.uniform(0.1, 1.0, size=(R, T_full)).astype(np.float32)[:, :T]
    return Workload(V, W.astype(np.float32), np.ascontiguousarray(H_init),
                    None, H0.astype(np.float32), {"config": 5})


def sparse_counts(N, T, density, seed, zipf=1.0, max_row_frac=0.3):
    """Term-document-like sparse counts with the structure of the sparse
    matrices of Sec. 4.2 (few nonzeros, a skewed number of them per row): row
    (term) n occurs in a number of columns (documents) proportional to
    rank^-zipf, the ranks a random permutation of the rows, scaled to the
    requested overall density and capped at max_row_frac * T; its columns are
    drawn uniformly without replacement; each count is 1 + Poisson(1.5).
    Returns (rows, cols, vals) in row order, vals float32."""
    rng = np.random.default_rng(seed)
    rank = rng.permutation(N) + 1.0
    w = rank ** -float(zipf)
    target, cap = density * N * T, float(int(max_row_frac * T))
    k = w / w.sum() * target
    for _ in range(50):                   # capped rows hand their excess to the others
        k = np.minimum(k, cap)
        free = k < cap
        deficit = target - k.sum()
        if deficit <= 0.5 or not free.any():
            break
        k[free] *= 1.0 + deficit / k[free].sum()
    k = np.rint(np.minimum(k, cap)).astype(np.int64)
    rows = np.repeat(np.arange(N, dtype=np.int64), k)
    cols = np.concatenate([rng.choice(T, size=int(kn), replace=False) for kn in k if kn > 0] or
                          [np.zeros(0, dtype=np.int64)]).astype(np.int64)
    vals = (1.0 + rng.poisson(1.5, size=rows.size)).astype(np.float32)
    return rows, cols, vals


def sparse_problem(N, T, R, density, seed, zipf=1.0):
    """A sparse-V parity problem: sparse_counts as a dense float32 V (the oracle's
    input) and uniform(0.1, 1) initial factors."""
    rows, cols, vals = sparse_counts(N, T, density, seed, zipf=zipf)
    V = np.zeros((N, T), dtype=np.float32)
    V[rows, cols] = vals
    rng = np.random.default_rng(seed + 7)
    W = rng.uniform(0.1, 1.0, size=(N, R)).astype(np.float32)
    H = rng.uniform(0.1, 1.0, size=(R, T)).astype(np.float32)
    return Workload(V, W, H, None, None, {"kind": "sparse", "seed": seed, "density": density, "zipf": zipf})


# Shapes of the paper's dense image matrices (Sec. 4.1): ORL 400 faces of 64 x 64
# pixels as a 4096 x 165 matrix (the shape the paper states), CMU PIE 11554
# faces of 32 x 32 pixels, 1024 x 11554.
PAPER_DENSE_SHAPES = {"orl": (4096, 165), "pie": (1024, 11554)}


def paper_dense(name, R):
    """Stand-in for a Sec. 4.1 image matrix at rank R: V = Poisson counts of a
    Gamma(0.5) product scaled to mean 60 (grey levels, few zeros), uniform
    initial factors (random_problem's recipe at the paper's shape)."""
    N, T = PAPER_DENSE_SHAPES[name]
    seed = DATA_SEED_BASE + 20 + sorted(PAPER_DENSE_SHAPES).index(name) * 10 + R
    return random_problem(N, T, R, seed, mean=60.0)


# Shapes of the paper's sparse matrices (Sec. 4.2): TDT2 36771 terms x 10212
# documents at 0.35% nonzeros, Newsgroup 61188 x 18774 at 0.2%.  The rank is not
# stated there; R = 40 is one of the ranks of its dense experiments.
SPARSE_SHAPES = {"tdt2": (36771, 10212, 0.0035), "newsgroup": (61188, 18774, 0.002)}


def sparse_workload(name, R=40):
    """(rows, cols, vals, N, T, W, H) of a synthetic stand-in for a Sec. 4.2
    matrix (no dense V is formed)."""
    N, T, density = SPARSE_SHAPES[name]
    seed = DATA_SEED_BASE + 10 + sorted(SPARSE_SHAPES).index(name)
    rows, cols, vals = sparse_counts(N, T, density, seed)
    rng = np.random.default_rng(seed + 1000)
    W = rng.uniform(0.1, 1.0, size=(N, R)).astype(np.float32)
    H = rng.uniform(0.1, 1.0, size=(R, T)).astype(np.float32)
    return rows, cols, vals, N, T, W, H


def config(k, **kw):
    return {1: config1, 2: config2, 3: config3, 4: config4, 5: config5}[k](**kw)
