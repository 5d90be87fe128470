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


def blobs(n: int, m: int, seed: int, spread: float = 1.5, n_test: int = 0):
    """Two isotropic Gaussian blobs with means +-1 on every axis.

    ceil(n/2) points carry label +1, the rest -1 (shuffled);
    x = y * 1 + spread * N(0, I).  With n_test > 0, a held-out set drawn
    the same way from the same stream follows (returned as a second pair).
    """
    rng = np.random.default_rng(seed)
    y = _balanced_labels(rng, n)
    X = y[:, None].astype(np.float64) + spread * rng.standard_normal((n, m))
    if n_test <= 0:
        return X.astype(np.float32), y
    yt = _balanced_labels(rng, n_test)
    Xt = yt[:, None].astype(np.float64) + spread * rng.standard_normal((n_test, m))
    return X.astype(np.float32), y, Xt.astype(np.float32), yt


def linear_teacher(n: int, m: int, seed: int, noise: float = 0.3, n_test: int = 0):
    """x ~ N(0, I); y = sign(w.x + noise * eps) with a unit-norm random w.
    With n_test > 0, held-out points of the same teacher follow."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, m))
    w = rng.standard_normal(m)
    w /= np.linalg.norm(w)
    s = X @ w + noise * rng.standard_normal(n)
    y = np.where(s >= 0.0, 1.0, -1.0).astype(np.float32)
    if n_test <= 0:
        return X.astype(np.float32), y
    Xt = rng.standard_normal((n_test, m))
    st = Xt @ w + noise * rng.standard_normal(n_test)
    yt = np.where(st >= 0.0, 1.0, -1.0).astype(np.float32)
    return X.astype(np.float32), y, Xt.astype(np.float32), yt


def covertype_like(n: int, m: int, seed: int, onehot_frac: float = 0.2,
                   n_centres: int = 50, flip: float = 0.05, n_test: int = 0):
    """Uniform [0,1] columns plus a one-hot block, labels from a random
    RBF teacher, then an exact fraction of label flips.

    The one-hot block has round(onehot_frac * m) columns, exactly one of
    which is 1 per row (category drawn uniformly).  The teacher is
    f(x) = sum_c beta_c exp(-0.5 ||x - z_c||^2) over n_centres data points
    z_c with beta ~ N(0, 1); y = sign(f - median f).  With n_test > 0,
    held-out points follow: same columns, same teacher and threshold, the
    same fraction of flips.
    """
    rng = np.random.default_rng(seed)
    n_hot = int(round(onehot_frac * m))
    n_cont = m - n_hot

    def draw(k):
        Z = np.zeros((k, m), dtype=np.float64)
        Z[:, :n_cont] = rng.random((k, n_cont))
        cat = rng.integers(0, n_hot, size=k)
        Z[np.arange(k), n_cont + cat] = 1.0
        return Z

    def teacher(Z):
        f = np.zeros(Z.shape[0])
        for c in range(n_centres):
            f += beta[c] * np.exp(-0.5 * ((Z - centres[c]) ** 2).sum(axis=1))
        return f

    def flipped(lab, k):
        idx = rng.choice(k, size=int(round(flip * k)), replace=False)
        lab[idx] = -lab[idx]
        return lab

    X = draw(n)
    centres = X[rng.choice(n, size=n_centres, replace=False)]
    beta = rng.standard_normal(n_centres)
    f = teacher(X)
    thr = np.median(f)
    y = flipped(np.where(f - thr >= 0.0, 1.0, -1.0), n)
    if n_test <= 0:
        return X.astype(np.float32), y.astype(np.float32)
    Xt = draw(n_test)
    yt = flipped(np.where(teacher(Xt) - thr >= 0.0, 1.0, -1.0), n_test)
    return X.astype(np.float32), y.astype(np.float32), Xt.astype(np.float32), yt.astype(np.float32)


def cluster_mixture(n: int, m: int, seed: int, per_class: int = 3, n_test: int = 0):
    """Balanced classes, each a mixture of `per_class` unit Gaussians whose
    centres are drawn from N(0, I); the cluster of a point is uniform.
    With n_test > 0, held-out points of the same mixture follow."""
    rng = np.random.default_rng(seed)
    centres = rng.standard_normal((2 * per_class, m))

    def draw(k_pts):
        lab = _balanced_labels(rng, k_pts)
        k = rng.integers(0, per_class, size=k_pts) + np.where(lab > 0, 0, per_class)
        return (centres[k] + rng.standard_normal((k_pts, m))).astype(np.float32), lab

    X, y = draw(n)
    if n_test <= 0:
        return X, y
    Xt, yt = draw(n_test)
    return X, y, Xt, yt


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


def holdout(name: str, n_test: int, n: int | None = None, seed: int | None = None):
    """The workload `name` (same training set as make_workload) and a
    held-out set of n_test points from the same generator and teacher."""
    wl = make_workload(name, n=n, seed=seed)
    gen = {"tiny": lambda k, s: blobs(k, 10, s, n_test=n_test),
           "letter": lambda k, s: linear_teacher(k, 100, s, n_test=n_test),
           "covertype": lambda k, s: covertype_like(k, 54, s, n_test=n_test),
           "large": lambda k, s: cluster_mixture(k, 20, s, n_test=n_test)}[name]
    seed0 = {"tiny": 0, "letter": 1, "covertype": 2, "large": 4}[name]
    X, y, Xt, yt = gen(wl.N, seed0 if seed is None else seed)
    assert np.array_equal(X, wl.X) and np.array_equal(y, wl.y)
    return wl, Xt, yt


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
