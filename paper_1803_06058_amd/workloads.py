"""Seeded synthetic workloads (inputs only; no GP arithmetic lives here).

The paper evaluates on UCI, airline and Bayesian-optimisation data that are not
available here; these generators stand in for them with the same kind of
structure: uniform inputs on the unit box, smooth sinusoidal targets plus
Gaussian noise, grids of m = 10^4 (1-D) up to 20^4 points, k = 50..100 Lanczos
steps, and s = 1000 samples at t = 10^4 test points (Sec. 4).

Draw order per problem (numpy PCG64, ``default_rng(seed)``): training x, target
noise, test x*; sampling noise z from ``default_rng(seed + 1)``.  Every array
is produced in float64 and rounded to the compute dtype once; the oracle is
fed the rounded values, so input quantisation is not counted as error.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np


@dataclass
class Problem:
    name: str
    d: int
    m: Tuple[int, ...]
    lo: Tuple[float, ...]
    hi: Tuple[float, ...]
    kernel: str
    lengthscale: Tuple[float, ...]
    outputscale: float
    noise: float
    k: int
    dtype: str                      # "f64" or "f32"
    x: np.ndarray                   # n x d
    y: np.ndarray                   # n
    xs: np.ndarray                  # t x d (variance queries)
    k_sample: int = 0
    xs_sample: Optional[np.ndarray] = None   # t_s x d
    z: Optional[np.ndarray] = None           # k_sample x s
    precision: str = "fp32"         # "fp64" | "fp32" | "bf16split"
    additive: bool = False          # sum of 1-D components (Sec. 3.4) instead of a product
    extra: Dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.x.shape[0]

    @property
    def t(self) -> int:
        return self.xs.shape[0]

    @property
    def np_dtype(self):
        return np.float64 if self.dtype == "f64" else np.float32


def _target(kind: str, x: np.ndarray) -> np.ndarray:
    if kind == "sin6":
        return np.sin(6 * np.pi * x[:, 0])
    if kind == "sin6_40":
        return np.sin(6 * np.pi * x[:, 0]) + 0.5 * np.sin(40 * np.pi * x[:, 0])
    if kind == "sincos4":
        return np.sin(4 * np.pi * x[:, 0]) * np.cos(4 * np.pi * x[:, 1])
    if kind == "sumsin":
        return sum(np.sin(2 * np.pi * x[:, i] * (i + 1)) for i in range(x.shape[1]))
    if kind == "styblinski_tang":
        # the additive Styblinski-Tang test function on [-5, 5]^d (x in [0, 1]^d
        # mapped there), divided by 40 to unit scale
        u = 10.0 * x - 5.0
        return 0.5 * np.sum(u ** 4 - 16.0 * u ** 2 + 5.0 * u, axis=1) / 40.0
    raise ValueError(kind)


def make_problem(name: str, *, d: int, n: int, m: Tuple[int, ...], kernel: str,
                 lengthscale: Tuple[float, ...], noise: float, k: int, t: int,
                 target: str, ynoise: float, dtype: str = "f32", precision: str = "fp32",
                 outputscale: float = 1.0, xs_linspace: bool = False, k_sample: int = 0,
                 t_sample: int = 0, s: int = 0, seed: int = 0, additive: bool = False) -> Problem:
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, size=(n, d))
    y = _target(target, x) + ynoise * rng.standard_normal(n)
    if xs_linspace:
        assert d == 1
        xs = np.linspace(0.0, 1.0, t)[:, None]
    else:
        xs = rng.uniform(0.0, 1.0, size=(t, d))
    xs_s = None
    z = None
    if k_sample > 0 and t_sample > 0:
        xs_s = rng.uniform(0.0, 1.0, size=(t_sample, d))
        z = np.random.default_rng(seed + 1).standard_normal((k_sample, s))
    npd = np.float64 if dtype == "f64" else np.float32
    cast = lambda a: None if a is None else np.ascontiguousarray(a.astype(npd))
    return Problem(name=name, d=d, m=tuple(m), lo=(0.0,) * d, hi=(1.0,) * d, kernel=kernel,
                   lengthscale=tuple(lengthscale), outputscale=outputscale, noise=noise, k=k,
                   dtype=dtype, x=cast(x), y=cast(y), xs=cast(xs), k_sample=k_sample,
                   xs_sample=cast(xs_s), z=cast(z), precision=precision, additive=additive)


# The five workloads.  `scale` < 1 shrinks n, t (and the 1-D grid) for tests
# that must finish quickly on the CPU oracle.
def config(idx: int, seed: int = 0, scale: float = 1.0, **over) -> Problem:
    def sc(v, lo=1):
        return max(lo, int(round(v * scale)))

    if idx == 1:
        kw = dict(d=1, n=1000, m=(100,), kernel="rbf", lengthscale=(0.1,), noise=0.01, k=50,
                  t=1000, target="sin6", ynoise=0.1, dtype="f64", precision="fp64",
                  xs_linspace=True)
        name = "c1_1d_fp64_n1000_m100_k50"
    elif idx == 2:
        kw = dict(d=1, n=sc(100_000), m=(sc(10_000, 8),), kernel="rbf", lengthscale=(0.02,),
                  noise=0.01, k=100, t=sc(1_000_000), target="sin6_40", ynoise=0.1,
                  dtype="f32", precision="fp32", k_sample=100, t_sample=sc(10_000), s=1000)
        name = "c2_1d_fp32_n1e5_m1e4_k100"
    elif idx == 3:
        mm = sc(128, 8)
        kw = dict(d=2, n=sc(500_000), m=(mm, mm), kernel="rbf", lengthscale=(0.05, 0.08),
                  noise=0.0025, k=100, t=sc(2_000_000), target="sincos4", ynoise=0.05,
                  dtype="f32", precision="bf16split")
        name = "c3_2d_bf16split_n5e5_m128x128_k100"
    elif idx == 4:
        mm = max(8, int(round(20 * scale ** 0.25)))
        kw = dict(d=4, n=sc(200_000), m=(mm,) * 4, kernel="matern52", lengthscale=(0.2,) * 4,
                  noise=0.01, k=64, t=sc(262_144), target="sumsin", ynoise=0.1, dtype="f32",
                  precision="fp32")
        name = "c4_4d_matern_n2e5_m20p4_k64"
    else:
        raise ValueError("config 5 is a batch; use batched_config()")
    kw.update(over)
    return make_problem(name, seed=seed, **kw)


# Additive composition (Sec. 3.4): one RBF component per dimension, 100 grid
# points each, as in the paper's additive Bayesian-optimisation model; the
# target is the (additive) Styblinski-Tang function.  d <= 4 here.
def additive_config(d: int = 4, n: int = 100_000, m: int = 100, k: int = 50, t: int = 1_000_000,
                    seed: int = 0, **over) -> Problem:
    kw = dict(d=d, n=n, m=(m,) * d, kernel="rbf", lengthscale=(0.15,) * d, noise=0.01, k=k, t=t,
              target="styblinski_tang", ynoise=0.1, dtype="f32", precision="fp32",
              additive=True)
    kw.update(over)
    return make_problem(f"add{d}d_n{n}_m{m}_k{k}", seed=seed, **kw)


def batched_config(G: int = 64, seed: int = 0, scale: float = 1.0, t_per_gp: int = 100_000,
                   n_lo: int = 2000, n_hi: int = 200_000) -> List[Problem]:
    """Many independent 1-D GPs of uneven size: n log-uniform on [n_lo, n_hi],
    m = clamp(n/10, 500, 20000), k in {50, 100}, lengthscale ~ U[0.01, 0.2],
    noise ~ U[0.001, 0.1], y = sin(2 pi f x) + N(0, 0.1^2), f ~ U[1, 20].
    Per-GP hyper-parameters are drawn first, then the data in GP order."""
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=G))
    ks = rng.choice([50, 100], size=G)
    ells = rng.uniform(0.01, 0.2, size=G)
    noises = rng.uniform(0.001, 0.1, size=G)
    fs = rng.uniform(1.0, 20.0, size=G)
    out = []
    for g in range(G):
        n = max(16, int(round(ns[g] * scale)))
        m = int(min(20000, max(500, n // 10)))
        if scale < 1.0:
            m = max(16, int(round(m * scale)))
        x = rng.uniform(0.0, 1.0, size=(n, 1))
        y = np.sin(2 * np.pi * fs[g] * x[:, 0]) + 0.1 * rng.standard_normal(n)
        t = max(1, int(round(t_per_gp * scale)))
        xs = rng.uniform(0.0, 1.0, size=(t, 1))
        f32 = lambda a: np.ascontiguousarray(a.astype(np.float32))
        out.append(Problem(name=f"c5_gp{g}", d=1, m=(m,), lo=(0.0,), hi=(1.0,), kernel="rbf",
                           lengthscale=(float(ells[g]),), outputscale=1.0, noise=float(noises[g]),
                           k=int(ks[g]), dtype="f32", x=f32(x), y=f32(y), xs=f32(xs),
                           precision="fp32"))
    return out
