"""Seeded synthetic LiNGAM data (the linear SEM of Sec. 2.2, Eq. (base_mat)).

X = B X + N with B strictly lower triangular in generation order and
independent, zero-mean, non-Gaussian noise N; the rows are then randomly
permuted so that the true causal order is not the row order.  This module
only generates inputs: it holds no part of the causal-order search, so both
the GPU library's tests/benchmark and the CPU oracle take their inputs from it.

Draw order for a generator `rng`:
  1. edge mask  rng.random((p, p)) < q        (strictly lower triangle kept)
  2. edge signs rng.choice([-1, 1], (p, p)) and magnitudes rng.uniform(lo, hi, (p, p))
  3. noise family per variable rng.integers(0, 3, p)   (only for noise="mixed")
  4. noise rows, variable by variable in generation order
  5. row permutation rng.permutation(p)
Seeds: numpy.random.default_rng([210913993, config, replicate]).
"""
from dataclasses import dataclass
from typing import Optional

import numpy as np

SEED_BASE = 2109_13993

# Unit-variance noise laws.  sign(g)|g|^1.5 has variance E|g|^3 = 2 sqrt(2/pi).
_POW15_SD = float(np.sqrt(2.0 * np.sqrt(2.0 / np.pi)))
NOISE_FAMILIES = ("uniform", "laplace", "power15")


@dataclass
class Dataset:
    X: np.ndarray          # p x n, row i = samples of variable i
    B: np.ndarray          # p x p, B[i, j] = weight of x_j in x_i (output indexing)
    true_order: np.ndarray  # a causal order (output indices), roots first
    perm: np.ndarray       # output row k is generation variable perm[k]
    noise: np.ndarray      # noise family index per output row (-1 = not from the 3 laws)


def rng_for(config: int, replicate: int = 0) -> np.random.Generator:
    return np.random.default_rng([SEED_BASE, int(config), int(replicate)])


def _noise_row(rng, family: str, n: int) -> np.ndarray:
    if family == "uniform":
        return rng.uniform(-np.sqrt(3.0), np.sqrt(3.0), n)
    if family == "laplace":
        return rng.laplace(0.0, 1.0 / np.sqrt(2.0), n)
    if family == "power15":
        g = rng.standard_normal(n)
        return np.sign(g) * np.abs(g) ** 1.5 / _POW15_SD
    if family == "gaussian":
        return rng.standard_normal(n)
    raise ValueError("unknown noise family %r" % family)


def _forward(B_gen: np.ndarray, E: np.ndarray) -> np.ndarray:
    """X = (I - B)^{-1} E for strictly lower-triangular B, by forward substitution."""
    p = B_gen.shape[0]
    X = np.empty_like(E)
    for i in range(p):
        row = E[i].copy()
        parents = np.nonzero(B_gen[i, :i])[0]
        for j in parents:
            row += B_gen[i, j] * X[j]
        X[i] = row
    return X


def lingam_dataset(p: int, n: int, q: float, noise: str = "uniform", rng=None,
                   weight_range=(0.5, 2.0), permute: bool = True,
                   dtype=np.float64) -> Dataset:
    """Random DAG with edge probability q, weights +-U[weight_range], and the
    given noise law ('uniform', 'laplace', 'power15', 'gaussian', or 'mixed' =
    one of the first three drawn per variable)."""
    if rng is None:
        rng = np.random.default_rng(0)
    mask = rng.random((p, p)) < q
    signs = rng.choice(np.array([-1.0, 1.0]), size=(p, p))
    mags = rng.uniform(weight_range[0], weight_range[1], size=(p, p))
    B_gen = np.tril(mask * signs * mags, k=-1)
    if noise == "mixed":
        fam = rng.integers(0, 3, p)
    else:
        fam = np.full(p, NOISE_FAMILIES.index(noise) if noise in NOISE_FAMILIES else -1)
    E = np.empty((p, n))
    for i in range(p):
        E[i] = _noise_row(rng, NOISE_FAMILIES[fam[i]] if fam[i] >= 0 else noise, n)
    X_gen = _forward(B_gen, E)
    perm = rng.permutation(p) if permute else np.arange(p)
    inv = np.empty(p, dtype=np.int64)
    inv[perm] = np.arange(p)
    X = np.ascontiguousarray(X_gen[perm]).astype(dtype, copy=False)
    B = B_gen[np.ix_(perm, perm)]
    return Dataset(X=X, B=B, true_order=inv.astype(np.int32), perm=perm, noise=fam[perm])


def order_respects_graph(order, B) -> bool:
    """True iff every edge j -> i of B (B[i, j] != 0) has j before i in `order`."""
    pos = np.empty(len(order), dtype=np.int64)
    pos[np.asarray(order)] = np.arange(len(order))
    ii, jj = np.nonzero(B)
    return bool(np.all(pos[jj] < pos[ii]))


# ---- the five benchmark workloads -------------------------------------------

def config_dataset(config: int, replicate: int = 0, dtype=np.float64) -> Dataset:
    """Workloads:
      1: p=10,   n=1000,  q=0.3,  uniform noise
      2: p=100,  n=10000, q=0.1,  noise law drawn per variable from the three laws
      3: p=500,  n=20000, q=0.02, Laplace noise
      4: p=100,  n=5000,  q=0.1,  mixed noise (base set for bootstrap resamples)
      5: p=1000, n=50000, q=0.01, uniform noise
    All with weights +-U[0.5, 2]."""
    spec = {
        1: (10, 1000, 0.3, "uniform"),
        2: (100, 10000, 0.1, "mixed"),
        3: (500, 20000, 0.02, "laplace"),
        4: (100, 5000, 0.1, "mixed"),
        5: (1000, 50000, 0.01, "uniform"),
    }[config]
    p, n, q, noise = spec
    return lingam_dataset(p, n, q, noise, rng=rng_for(config, replicate), dtype=dtype)


def bootstrap_indices(n: int, count: int, rng) -> np.ndarray:
    """count x n sample indices drawn with replacement."""
    return rng.integers(0, n, size=(count, n), dtype=np.int64)


def uneven_datasets(count: int = 64, rng=None, p_range=(20, 200), n_range=(1000, 20000),
                    q: float = 0.1, noise: str = "mixed"):
    """Independent datasets of uneven (p, n): p ~ U{p_range}, n ~ U{n_range}."""
    if rng is None:
        rng = rng_for(4, 1)
    out = []
    for _ in range(count):
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        out.append(lingam_dataset(p, n, q, noise, rng=rng))
    return out


def paper_scalability_dataset(p: int, n: int, dense: bool, rng) -> Dataset:
    """The scalability workload of Sec. 5.4: parents per variable U[1, 0.2p]
    (sparse) or U[0.25p, 0.5p] (dense), weights +-U[0.5, 0.95], noise
    sign(g)|g|^e with e ~ U([0.5, 0.8] u [1.2, 2]), rows permuted.

    The paper does not say how the variables are scaled.  Summed over up to
    0.5p parents with weights near 1, the variances would grow geometrically
    along the order until the deep variables are exact linear functions of
    their parents in binary64; so each variable is scaled to unit sample
    variance once it is generated, before its children are formed (its row
    of B and its noise are scaled with it, so X = B X + N still holds)."""
    lo, hi = (1, max(1, int(0.2 * p))) if not dense else (max(1, int(0.25 * p)), max(1, int(0.5 * p)))
    B_gen = np.zeros((p, p))
    for i in range(1, p):
        k = min(i, int(rng.integers(lo, hi + 1)))
        par = rng.choice(i, size=k, replace=False)
        B_gen[i, par] = rng.choice([-1.0, 1.0], size=k) * rng.uniform(0.5, 0.95, size=k)
    E = np.empty((p, n))
    for i in range(p):
        e = rng.uniform(0.5, 0.8) if rng.random() < 0.5 else rng.uniform(1.2, 2.0)
        g = rng.standard_normal(n)
        E[i] = np.sign(g) * np.abs(g) ** e
    X_gen = np.empty((p, n))
    for i in range(p):
        row = E[i] + B_gen[i, :i] @ X_gen[:i] if i > 0 else E[i].copy()
        s = row.std(ddof=1)
        X_gen[i] = row / s
        B_gen[i] /= s
    perm = rng.permutation(p)
    inv = np.empty(p, dtype=np.int64)
    inv[perm] = np.arange(p)
    return Dataset(X=np.ascontiguousarray(X_gen[perm]), B=B_gen[np.ix_(perm, perm)],
                   true_order=inv.astype(np.int32), perm=perm, noise=np.full(p, -1))


# ---- stand-ins for the paper's metabolic-flux data sets (Sec. 5.2) ---------------

# p of the real data sets of the paper's Table 1 (their n is 10000)
FLUX_P = {"ecoli_core": 85, "iJR904": 770, "iAF1260b": 1588, "iAF1260": 1633, "iY75_1357": 2249,
          "iECDH10B_1368": 2252, "iML1515": 2326, "iEC1372_W3110": 2339}


def flux_like_dataset(p: int, n: int, rng, noise: float = 1e-3, met_frac: float = 0.4) -> Dataset:
    """Rows shaped like sampled fluxes of a metabolic network: the p
    reactions' flux samples lie (up to relative `noise`) in the null space of
    a sparse stoichiometric-like matrix S (m = met_frac p metabolites; each
    reaction consumes or produces 1 to 3 of them with coefficients in
    {+-1, +-2}).  v = N z, N an orthonormal basis of null(S) and z
    non-Gaussian (uniform) coordinates, so the variables are strongly and
    jointly collinear; with noise = 0 they are exactly linearly dependent
    (p - rank S degrees of freedom, and reactions outside every null vector
    carry no flux at all), which the search must report as degenerate.
    The real data sets are not available; only their shape (p, n) and the
    collinearity of steady-state fluxes are reproduced."""
    m = max(1, int(round(met_frac * p)))
    S = np.zeros((m, p))
    for j in range(p):
        k = int(rng.integers(1, 4))
        rows = rng.choice(m, size=k, replace=False)
        S[rows, j] = rng.choice(np.array([-2.0, -1.0, 1.0, 2.0]), size=k)
    _, sv, Vt = np.linalg.svd(S, full_matrices=True)
    rank = int(np.sum(sv > 1e-10 * sv[0]))
    N = Vt[rank:].T                                   # p x (p - rank), orthonormal
    z = rng.uniform(-np.sqrt(3.0), np.sqrt(3.0), (N.shape[1], n))
    X = N @ z
    if noise > 0:
        # blocked reactions (rows that are zero in the null space) get noise
        # at the scale of a typical row
        sd = X.std(axis=1, keepdims=True)
        sd = np.maximum(sd, np.median(sd))
        X += noise * sd * rng.laplace(0.0, 1.0 / np.sqrt(2.0), (p, n))
    return Dataset(X=np.ascontiguousarray(X), B=np.zeros((p, p)), true_order=np.arange(p, dtype=np.int32),
                   perm=np.arange(p), noise=np.full(p, -1))
