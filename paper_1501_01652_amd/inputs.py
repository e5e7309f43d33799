"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds random-number generation only: none of the arithmetic of the
method lives here.  The coefficient distributions follow the paper's numerical
experiments (independent Gaussians, Sec. 5.3 and Sec. 6.1) and the workload
definitions of the three tasks.
"""
from __future__ import annotations

import numpy as np

SEED_SCHLOMILCH = 150101
SEED_FOURIER_BESSEL = 150102
SEED_DHT0 = 150103
SEED_BATCH = 150104
SEED_SERVE = 150105
SEED_SAMPLED_ROWS = 150106


def coefficients(kind: str, N: int, seed: int) -> np.ndarray:
    """c_n, n = 1..N, as FP64.

    kind: 'uniform'  c_n iid Uniform[-1, 1]
          'gauss'    c_n iid N(0, 1)
          'decay'    c_n = n^(-1/2) * N(0, 1)
    """
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.uniform(-1.0, 1.0, N)
    if kind == "gauss":
        return rng.standard_normal(N)
    if kind == "decay":
        n = np.arange(1, N + 1, dtype=np.float64)
        return rng.standard_normal(N) / np.sqrt(n)
    raise ValueError(kind)


def workload(task: str, N: int | None = None, seed: int | None = None) -> np.ndarray:
    """The coefficient vector of each task's standard synthetic workload."""
    if task == "schlomilch":
        return coefficients("uniform", N or 4096, SEED_SCHLOMILCH if seed is None else seed)
    if task == "fourier_bessel":
        return coefficients("decay", N or 2 ** 16, SEED_FOURIER_BESSEL if seed is None else seed)
    if task == "dht0":
        return coefficients("gauss", N or 2 ** 20, SEED_DHT0 if seed is None else seed)
    raise ValueError(task)


def sampled_rows(N: int, count: int, boundaries=(), seed: int = SEED_SAMPLED_ROWS) -> np.ndarray:
    """A sorted set of 1-based row indices: the first rows, the last rows, a
    band of +-2 around each given boundary row, and uniform random rows."""
    rng = np.random.default_rng(seed)
    rows = set(range(1, min(N, 16) + 1)) | set(range(max(1, N - 3), N + 1))
    for b in boundaries:
        for d in range(-2, 3):
            if 1 <= b + d <= N:
                rows.add(int(b + d))
    while len(rows) < min(count, N):
        rows.add(int(rng.integers(1, N + 1)))
    return np.array(sorted(rows), dtype=np.int64)


TASK_MIX = (("schlomilch", 0.4), ("fourier_bessel", 0.4), ("dht0", 0.2))
EPS_SET = (1e-4, 1e-8, 1e-14)


def batch_specs(count: int = 1024, seed: int = SEED_BATCH, nlo: int = 2 ** 8, nhi: int = 2 ** 16,
                rhs_max: int = 64):
    """Request specs of the batched workload: task 40/40/20 (Schlomilch,
    Fourier-Bessel, DHT), N log-uniform in [nlo, nhi], 1..rhs_max right-hand
    sides, eps from {1e-4, 1e-8, 1e-14}, and a per-request seed for c ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    names = [t for t, _ in TASK_MIX]
    probs = [p for _, p in TASK_MIX]
    specs = []
    for i in range(count):
        specs.append({"task": names[int(rng.choice(3, p=probs))],
                      "N": int(np.exp(rng.uniform(np.log(nlo), np.log(nhi)))),
                      "nrhs": int(rng.integers(1, rhs_max + 1)),
                      "eps": float(EPS_SET[int(rng.integers(0, 3))]),
                      "seed": int(seed * 10007 + i)})
    return specs


def serve_trace(rate: float = 2000.0, seconds: float = 60.0, seed: int = SEED_SERVE,
                lg_lo: int = 10, lg_hi: int = 22):
    """Open-loop Poisson arrivals at `rate` per second for `seconds`: the same
    task and eps mix, one right-hand side, N log-uniform over the integers
    [2^lg_lo, 2^lg_hi] (so that most large sizes are seen once)."""
    rng = np.random.default_rng(seed)
    names = [t for t, _ in TASK_MIX]
    probs = [p for _, p in TASK_MIX]
    t, out = 0.0, []
    lo, hi = np.log(2.0 ** lg_lo), np.log(2.0 ** lg_hi + 1.0)
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= seconds:
            break
        out.append({"arrival": t, "task": names[int(rng.choice(3, p=probs))],
                    "N": int(min(2 ** lg_hi, np.exp(rng.uniform(lo, hi)))),
                    "eps": float(EPS_SET[int(rng.integers(0, 3))])})
    return out
