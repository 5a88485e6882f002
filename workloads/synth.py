"""Seeded synthetic inputs for dense CP decomposition workloads.

Every array is drawn on the host in float64 with ``numpy.random.default_rng`` and only cast
afterwards, so a test and the benchmark see the same values for the same seed.

Seed convention: problem ``i`` of workload ``c`` uses seed ``1000*c + i`` for the planted
factors and noise, and ``1000*c + i + 500`` for the initial guess.

The planted tensor X = [[B(1), ..., B(N)]] is the input of the method, not a step of it; it is
formed here as one matrix product of the mode-1 unfolding with the Khatri-Rao product of the
remaining factors, which keeps input generation fast at 400^3.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "seed_for",
    "gaussian_factors",
    "uniform_factors",
    "congruent_factors",
    "lognorm_factors",
    "planted_tensor",
    "add_noise",
    "Problem",
    "make_problem",
    "WORKLOADS",
    "batched_problems",
    "bf16_round",
    "bf16_planes",
    "bf16_values",
]


def seed_for(workload: int, problem: int = 0, init: bool = False) -> int:
    return 1000 * workload + problem + (500 if init else 0)


def gaussian_factors(dims, rank, rng):
    """Factor matrices with i.i.d. N(0,1) entries, one [s_n, R] array per mode."""
    return [rng.standard_normal((int(s), int(rank))) for s in dims]


def uniform_factors(dims, rank, rng, lo=0.0, hi=1.0):
    """Factor matrices with i.i.d. U(lo, hi) entries."""
    return [rng.uniform(lo, hi, size=(int(s), int(rank))) for s in dims]


def congruent_factors(dims, rank, rng, cosine=0.9):
    """Factors whose columns have pairwise cosine exactly ``cosine`` in every mode.

    A = sqrt(s) * Q * L^T, where Q holds orthonormal columns (QR of a Gaussian matrix) and
    L L^T = C = (1 - cosine) I + cosine * 1 1^T, so that A^T A = s * C.
    """
    c = (1.0 - cosine) * np.eye(rank) + cosine * np.ones((rank, rank))
    low = np.linalg.cholesky(c)
    out = []
    for s in dims:
        if s < rank:
            raise ValueError("congruent factors need s_n >= R")
        q, _ = np.linalg.qr(rng.standard_normal((int(s), int(rank))))
        out.append(np.sqrt(float(s)) * q @ low.T)
    return out


def lognorm_factors(dims, rank, rng, lo=1.0, hi=100.0):
    """Gaussian columns normalised to unit length, then scaled by 10^U(log10 lo, log10 hi)
    independently for every (mode, component)."""
    out = []
    for s in dims:
        a = rng.standard_normal((int(s), int(rank)))
        a /= np.linalg.norm(a, axis=0, keepdims=True)
        a *= 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size=(1, int(rank)))
        out.append(a)
    return out


def planted_tensor(factors):
    """Dense C-order tensor with exactly the CP structure of ``factors`` (float64)."""
    dims = [f.shape[0] for f in factors]
    rank = factors[0].shape[1]
    rest = np.ones((1, rank))
    for f in factors[1:]:
        rest = (rest[:, None, :] * f[None, :, :]).reshape(-1, rank)
    return (factors[0] @ rest.T).reshape(dims)


def add_noise(x, eta, rng):
    """X + eta * ||X||_F * E / ||E||_F with E i.i.d. N(0,1)."""
    if eta == 0.0:
        return x
    e = rng.standard_normal(x.shape)
    return x + eta * np.linalg.norm(x) * e / np.linalg.norm(e)


@dataclass
class Problem:
    """A dense tensor to decompose plus its planted factors and an initial guess (all float64)."""

    x: np.ndarray
    planted: list
    init: list
    rank: int
    meta: dict = field(default_factory=dict)

    @property
    def dims(self):
        return tuple(self.x.shape)


def make_problem(dims, rank, workload=0, problem=0, kind="gaussian", noise=0.0, init_rank=None,
                 cosine=0.9):
    """Build one seeded problem.

    kind: "gaussian" (N(0,1) factors), "uniform01", "uniform11", "congruent" (pairwise column
    cosine ``cosine``), "lognorm" (unit columns scaled log-uniformly over [1, 100]).
    The initial guess is N(0,1) with rank ``init_rank`` (default ``rank``).
    """
    rng = np.random.default_rng(seed_for(workload, problem))
    if kind == "gaussian":
        fac = gaussian_factors(dims, rank, rng)
    elif kind == "uniform01":
        fac = uniform_factors(dims, rank, rng, 0.0, 1.0)
    elif kind == "uniform11":
        fac = uniform_factors(dims, rank, rng, -1.0, 1.0)
    elif kind == "congruent":
        fac = congruent_factors(dims, rank, rng, cosine)
    elif kind == "lognorm":
        fac = lognorm_factors(dims, rank, rng)
    else:
        raise ValueError(kind)
    x = add_noise(planted_tensor(fac), noise, rng)
    irng = np.random.default_rng(seed_for(workload, problem, init=True))
    init = gaussian_factors(dims, init_rank or rank, irng)
    return Problem(x=x, planted=fac, init=init, rank=rank,
                   meta=dict(kind=kind, noise=noise, workload=workload, problem=problem))


def batched_problems(count=64, workload=5, lo=60, hi=200, ranks=(8, 16, 32, 64), noise=1e-4):
    """Workload 5: `count` independent problems of order 3 with mode sizes drawn uniformly from
    [lo, hi] per mode and the rank drawn from `ranks`, N(0,1) planted factors, relative noise
    `noise`. The shape of problem i comes from seed seed_for(workload, i, init=True) + 1, its data
    from make_problem(..., workload, i)."""
    out = []
    for i in range(count):
        srng = np.random.default_rng(seed_for(workload, i, init=True) + 1)
        dims = tuple(int(v) for v in srng.integers(lo, hi + 1, size=3))
        rank = int(srng.choice(ranks))
        out.append(make_problem(dims, rank, workload=workload, problem=i, noise=noise))
    return out


def bf16_round(x):
    """Bits of float32(x) rounded to the nearest bfloat16, ties to even (finite values): the
    storage format of the bfloat16 tensor forms. Returns a uint16 array."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    return ((u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) >> np.uint32(16)).astype(np.uint16)


def _bf16_to_f32(h):
    return (h.astype(np.uint32) << np.uint32(16)).view(np.float32)


def bf16_planes(x, split=False):
    """Storage of tensor x as bfloat16: the rounded values (hi) and, with split=True, the rounded
    remainder lo = bf16(float32(x) - hi) as a second plane, stacked as (2, *shape)."""
    x32 = np.ascontiguousarray(x, dtype=np.float32)
    hi = bf16_round(x32)
    if not split:
        return hi
    lo = bf16_round(x32 - _bf16_to_f32(hi))
    return np.stack([hi, lo])


def bf16_values(planes, split=False):
    """The float64 tensor a bfloat16 storage represents: hi, or hi + lo for a split (2, ...)
    array."""
    v = _bf16_to_f32(np.asarray(planes)).astype(np.float64)
    return v[0] + v[1] if split else v


# The five workloads: (dims, rank, kind, noise, storage dtype).
WORKLOADS = {
    1: dict(dims=(40, 40, 40), rank=5, kind="gaussian", noise=0.0, dtype="f64"),
    2: dict(dims=(300, 300, 300), rank=50, kind="congruent", noise=1e-6, dtype="f64"),
    3: dict(dims=(400, 400, 400), rank=100, kind="gaussian", noise=0.0, dtype="f32"),
    4: dict(dims=(80, 80, 80, 80), rank=64, kind="lognorm", noise=1e-3, dtype="bf16"),
    5: dict(dims="64 problems, each mode U{60..200}", rank="U{8,16,32,64}", kind="gaussian",
            noise=1e-4, dtype="f32"),
}
