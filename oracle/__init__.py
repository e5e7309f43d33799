"""CPU oracle for f_k = sum_n c_n J_0(r_k w_n) -- TEST INFRASTRUCTURE ONLY.

Plain FP64 direct summation (the definition of the sums, Sec. 1 eq. (2) of
Townsend's "A fast analysis-based discrete Hankel transform using asymptotic
expansions"), with its own J_0 (Taylor series, Sec. 3.2, in double-double for
z < 20; Hankel expansion, Sec. 3.1, with exact phase reduction otherwise) and its
own Bessel roots (regula falsi inside the bracket of Lemma 3.2).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never does, and this
package imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hank_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

TASKS = {"schlomilch": 0, "fourier_bessel": 1, "dht0": 2,
         "schlomilch_paper_grid": 3, "fourier_bessel_paper_grid": 4}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, no GPU)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fPIC",
               "-shared", "-o", tmp, _SRC, "-lm", "-lpthread"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build()
            lib = ctypes.CDLL(_LIB)
            d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
            p = ctypes.c_void_p
            lib.or_j0.restype = d
            lib.or_j0.argtypes = [d]
            lib.or_j1.restype = d
            lib.or_j1.argtypes = [d]
            lib.or_y0.restype = d
            lib.or_y0.argtypes = [d]
            lib.or_y1.restype = d
            lib.or_y1.argtypes = [d]
            lib.or_j0_phase.restype = d
            lib.or_j0_phase.argtypes = [i64, i64, d, d]
            lib.or_root_offsets.restype = i64
            lib.or_root_offsets.argtypes = [i64, p]
            lib.or_eval_rows.restype = i32
            lib.or_eval_rows.argtypes = [i32, i64, p, p, i64, p, p, i32]
            lib.or_entry.restype = d
            lib.or_entry.argtypes = [i32, i64, p, i64, i64]
            lib.or_default_threads.restype = i32
            lib.or_hankel_j0.restype = d
            lib.or_hankel_j0.argtypes = [d, i32]
            lib.or_jn.restype = d
            lib.or_jn.argtypes = [i32, d]
            lib.or_eval_rows_nu.restype = i32
            lib.or_eval_rows_nu.argtypes = [i32, i32, i64, i64, p, p, i64, p, p, i32]
            lib.or_entry_nu.restype = d
            lib.or_entry_nu.argtypes = [i32, i32, i64, i64, p, i64, i64]
            lib.or_dht_weights.restype = None
            lib.or_dht_weights.argtypes = [i64, p, p]
            _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def j0(z):
    lib = _load()
    return np.array([lib.or_j0(float(x)) for x in np.atleast_1d(z)])


def j1(z):
    lib = _load()
    return np.array([lib.or_j1(float(x)) for x in np.atleast_1d(z)])


def y0(z):
    lib = _load()
    return np.array([lib.or_y0(float(x)) for x in np.atleast_1d(z)])


def y1(z):
    lib = _load()
    return np.array([lib.or_y1(float(x)) for x in np.atleast_1d(z)])


def hankel_j0(z: float, M: int) -> float:
    """The first 2M terms of the Hankel expansion of J_0 (Sec. 3.1)."""
    return _load().or_hankel_j0(float(z), int(M))


def j0_phase(I: int, D: int, delta_hi: float = 0.0, delta_lo: float = 0.0) -> float:
    """J_0(pi*I/D + delta) with the phase reduced exactly."""
    return _load().or_j0_phase(int(I), int(D), float(delta_hi), float(delta_lo))


_root_cache: dict = {}


def root_offsets(nmax: int) -> np.ndarray:
    """b_n = j_{0,n} - (n - 1/4) pi for n = 1..nmax (Lemma 3.2)."""
    nmax = int(nmax)
    for have, arr in _root_cache.items():
        if have >= nmax:
            return arr[:nmax].copy()
    out = np.empty(nmax, dtype=np.float64)
    bad = _load().or_root_offsets(nmax, _ptr(out))
    if bad:
        raise RuntimeError("oracle root bracket failed for %d roots" % bad)
    _root_cache.clear()
    _root_cache[nmax] = out
    return out.copy()


def roots(nmax: int) -> np.ndarray:
    n = np.arange(1, nmax + 1, dtype=np.float64)
    return (n - 0.25) * np.pi + root_offsets(nmax)


def default_threads() -> int:
    return int(_load().or_default_threads())


def jn(nu: int, z):
    """J_nu(z) for integer 0 <= nu <= 12 (elementwise)."""
    lib = _load()
    return np.array([lib.or_jn(int(nu), float(x)) for x in np.atleast_1d(z)])


def eval_rows(task: str, c: np.ndarray, rows=None, nthreads: int = 0, nu: int = 0,
              shift: int = 0) -> np.ndarray:
    """f_k for the 1-based ``rows`` (all rows when None) by direct summation;
    for the Schlomilch and Fourier-Bessel tasks optionally of order nu, and for
    the Schlomilch tasks with w_n = (n + shift) pi."""
    lib = _load()
    c = np.ascontiguousarray(c, dtype=np.float64)
    N = c.shape[0]
    t = TASKS[task]
    b = None
    if t in (1, 2, 4):
        b = root_offsets(N + 1)
    if rows is None:
        rows = np.arange(1, N + 1, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    out = np.empty(rows.shape[0], dtype=np.float64)
    rc = lib.or_eval_rows_nu(t, int(nu), int(shift), N, _ptr(c), _ptr(b), rows.shape[0], _ptr(rows),
                             _ptr(out), int(nthreads))
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return out


def dht_weights(N: int) -> np.ndarray:
    """v_n = 2 / J_1(j_{0,n})^2 for n = 1..N (Sec. 6, eq. (selfinverse))."""
    out = np.empty(int(N), dtype=np.float64)
    _load().or_dht_weights(int(N), _ptr(root_offsets(N)), _ptr(out))
    return out


def dht0_inverse_rows(f: np.ndarray, rows=None, nthreads: int = 0) -> np.ndarray:
    """c_k = (v_k / j_{0,N+1}^2) sum_n J_0(j_{0,k} j_{0,n} / j_{0,N+1}) v_n f_n for
    the 1-based ``rows`` (eq. (inverseTest) applied to f): the DHT's direct sum
    between the two diagonal scalings."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    N = f.shape[0]
    v = dht_weights(N)
    S = roots(N + 1)[-1]
    if rows is None:
        rows = np.arange(1, N + 1, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    g = eval_rows("dht0", v * f, rows=rows, nthreads=nthreads)
    return v[rows - 1] * g / (S * S)


def entry(task: str, N: int, k: int, n: int, nu: int = 0, shift: int = 0) -> float:
    """J_nu(r_k w_n) for one matrix entry (nu: not the DHT; shift: Schlomilch only)."""
    t = TASKS[task]
    b = root_offsets(N + 1) if t in (1, 2, 4) else None
    return _load().or_entry_nu(t, int(nu), int(shift), int(N), _ptr(b), int(k), int(n))
