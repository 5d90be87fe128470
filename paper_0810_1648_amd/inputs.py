"""Seeded synthetic training sets shaped like the paper's workloads.

This module only draws data: features X (float32, N x m, row-major) and
labels y (float32, +-1), plus the hyper-parameters each workload is run
with.  It holds none of the solver's arithmetic, so both the FP64 oracle
and the HIP path consume the very same arrays.

The paper evaluates on UCI sets, Covertype and MNIST (Tables 1-3), none of
which are available here.  The generators below stand in for their shapes
(sizes, dimensionality, one-hot columns, label noise); no record of those
datasets is reproduced.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    """One training problem: data plus the parameters it is solved with."""

    name: str
    X: np.ndarray            # (N, m) float32, row-major
    y: np.ndarray            # (N,) float32 in {-1, +1}
    gamma: float             # RBF width: K(x, z) = exp(-gamma ||x - z||^2)
    C: float                 # soft-margin cost; adds 1/C to the diagonal
    lam: float               # bias augmentation constant (lambda)
    delta: float = 0.1       # diagonal-dominance margin of the weighting rule
    precision: str = "fp32"  # "fp64" | "fp32" | "mixed"
    tol_abs: float = 0.0
    tol_rel: float = 1e-7
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.X.shape[0])

    @property
    def m(self) -> int:
        return int(self.X.shape[1])


def _balanced_labels(rng: np.random.Generator, n: int) -> np.ndarray:
    y = np.ones(n, dtype=np.float32)
    y[(n + 1) // 2:] = -1.0
    rng.shuffle(y)
    return y


def blobs(n: int, m: int, seed: int, spread: float = 1.5):
    """Two isotropic Gaussian blobs with means +-1 on every axis.

    ceil(n/2) points carry label +1, the rest -1 (shuffled);
    x = y * 1 + spread * N(0, I).
    """
    rng = np.random.default_rng(seed)
    y = _balanced_labels(rng, n)
    X = y[:, None].astype(np.float64) + spread * rng.standard_normal((n, m))
    return X.astype(np.float32), y


def linear_teacher(n: int, m: int, seed: int, noise: float = 0.3):
    """x ~ N(0, I); y = sign(w.x + noise * eps) with a unit-norm random w."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, m))
    w = rng.standard_normal(m)
    w /= np.linalg.norm(w)
    s = X @ w + noise * rng.standard_normal(n)
    y = np.where(s >= 0.0, 1.0, -1.0).astype(np.float32)
    return X.astype(np.float32), y


def covertype_like(n: int, m: int, seed: int, onehot_frac: float = 0.2,
                   n_centres: int = 50, flip: float = 0.05):
    """Uniform [0,1] columns plus a one-hot block, labels from a random
    RBF teacher, then an exact fraction of label flips.

    The one-hot block has round(onehot_frac * m) columns, exactly one of
    which is 1 per row (category drawn uniformly).  The teacher is
    f(x) = sum_c beta_c exp(-0.5 ||x - z_c||^2) over n_centres data points
    z_c with beta ~ N(0, 1); y = sign(f - median f).
    """
    rng = np.random.default_rng(seed)
    n_hot = int(round(onehot_frac * m))
    n_cont = m - n_hot
    X = np.zeros((n, m), dtype=np.float64)
    X[:, :n_cont] = rng.random((n, n_cont))
    cat = rng.integers(0, n_hot, size=n)
    X[np.arange(n), n_cont + cat] = 1.0
    centres = X[rng.choice(n, size=n_centres, replace=False)]
    beta = rng.standard_normal(n_centres)
    f = np.zeros(n)
    for c in range(n_centres):
        f += beta[c] * np.exp(-0.5 * ((X - centres[c]) ** 2).sum(axis=1))
    y = np.where(f - np.median(f) >= 0.0, 1.0, -1.0)
    flip_idx = rng.choice(n, size=int(round(flip * n)), replace=False)
    y[flip_idx] = -y[flip_idx]
    return X.astype(np.float32), y.astype(np.float32)


def cluster_mixture(n: int, m: int, seed: int, per_class: int = 3):
    """Balanced classes, each a mixture of `per_class` unit Gaussians whose
    centres are drawn from N(0, I); the cluster of a point is uniform."""
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((2 * per_class, m))
    y = _balanced_labels(rng, n)
    k = rng.integers(0, per_class, size=n) + np.where(y > 0, 0, per_class)
    X = centres[k] + rng.standard_normal((n, m))
    return X.astype(np.float32), y


# The five workloads.  Sizes, dimensions and hyper-parameters of the
# paper-shaped configurations; `n` may be overridden for scaled-down runs of
# the same recipe.
def make_workload(name: str, n: int | None = None, seed: int | None = None) -> Workload:
    if name == "tiny":            # smallest UCI-sized problem, FP64
        n = 500 if n is None else n
        seed = 0 if seed is None else seed
        X, y = blobs(n, 10, seed)
        return Workload(name, X, y, gamma=0.1, C=1.0, lam=1.0 / n,
                        precision="fp64", tol_abs=1e-8, tol_rel=0.0)
    if name == "letter":          # N = 20k, m = 100, plain FP32, K' materialised
        n = 20000 if n is None else n
        seed = 1 if seed is None else seed
        X, y = linear_teacher(n, 100, seed)
        return Workload(name, X, y, gamma=1.0 / 100, C=10.0, lam=1.0 / n,
                        precision="fp32", tol_rel=1e-7)
    if name == "covertype":       # N = 100k, m = 54, mixed vs plain FP32
        n = 100000 if n is None else n
        seed = 2 if seed is None else seed
        X, y = covertype_like(n, 54, seed)
        return Workload(name, X, y, gamma=0.5, C=1.0, lam=1.0 / n,
                        precision="mixed", tol_rel=1e-7)
    if name == "large":           # N = 300k, m = 20, K' recomputed per tile
        n = 300000 if n is None else n
        seed = 4 if seed is None else seed
        X, y = cluster_mixture(n, 20, seed)
        return Workload(name, X, y, gamma=0.05, C=1.0, lam=1.0 / n,
                        precision="mixed", tol_rel=1e-7)
    raise ValueError(f"unknown workload {name!r}")


@dataclass
class Request:
    """One solve request of the serving stream."""

    rid: int
    arrival_s: float
    workload: Workload


def serving_stream(n_requests: int = 512, rate_per_s: float = 10.0, seed: int = 3,
                   n_min: int = 1000, n_max: int = 16000):
    """Poisson stream of SVM solves of uneven size.

    N is log-uniform in [n_min, n_max], m uniform in {8, 32, 128}, C uniform
    in {0.1, 1, 10}; each request's data are two blobs as in the tiny
    workload with seed 1000 + request id; gamma = 1/m, tol_rel = 1e-7.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        n = int(math.floor(math.exp(rng.uniform(math.log(n_min), math.log(n_max)))))
        m = int(rng.choice([8, 32, 128]))
        C = float(rng.choice([0.1, 1.0, 10.0]))
        X, y = blobs(n, m, 1000 + r)
        wl = Workload(f"req{r}", X, y, gamma=1.0 / m, C=C, lam=1.0 / n,
                      precision="fp32", tol_rel=1e-7)
        out.append(Request(r, t, wl))
    return out


def random_spd_dominant(n: int, seed: int, margin: float = 0.5, density: float = 1.0):
    """Random symmetric matrix with a strictly dominant positive diagonal.

    Off-diagonal entries ~ U(-1, 1) (kept with probability `density`);
    A_ii = (1 + margin) * sum_j |A_ij| + 1e-3.  Returned in float64.
    """
    rng = np.random.default_rng(seed)
    B = rng.uniform(-1.0, 1.0, size=(n, n))
    if density < 1.0:
        B *= rng.random((n, n)) < density
    A = np.triu(B, 1)
    A = A + A.T
    A[np.diag_indices(n)] = (1.0 + margin) * np.abs(A).sum(axis=1) + 1e-3
    return A


def chain_matrix(n: int, seed: int):
    """Random tridiagonal (tree-structured) symmetric positive definite matrix."""
    rng = np.random.default_rng(seed)
    off = rng.uniform(-1.0, 1.0, size=n - 1)
    A = np.diag(off, 1) + np.diag(off, -1)
    A[np.diag_indices(n)] = np.abs(A).sum(axis=1) + rng.uniform(0.2, 1.0, size=n)
    return A


def equicorrelated(n: int, diag: float, off: float):
    """A = off * (ones - I) + diag * I."""
    A = np.full((n, n), float(off))
    A[np.diag_indices(n)] = float(diag)
    return A
