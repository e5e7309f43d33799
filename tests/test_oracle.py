"""Pins for the CPU oracle (test infrastructure) against values fixed by the
paper and by independent mathematics: mpmath's arbitrary-precision Bessel
functions and zeros, the Wronskian identity, the Lemma 3.2 root bracket, the
remainder claim of Sec. 3.1, and brute-force high-precision sums."""
import math

import mpmath
import numpy as np
import pytest

import oracle

mpmath.mp.dps = 40


def mp_j0(z):
    return float(mpmath.besselj(0, z))


def test_j0_special_values():
    assert oracle.j0(0.0)[0] == 1.0
    # j_{0,1} ~ 2.404825557695773: J_0 vanishes there to rounding
    assert abs(oracle.j0(2.404825557695773)[0]) < 1e-15
    r = oracle.roots(1)[0]
    assert abs(r - 2.404825557695773) < 4e-16


def test_j0_against_mpmath_dense():
    rng = np.random.default_rng(1)
    zs = np.concatenate([rng.uniform(0, 30, 300), rng.uniform(30, 400, 100),
                         10.0 ** rng.uniform(2.5, 6.6, 100), [19.999999, 20.0, 20.000001]])
    got = oracle.j0(zs)
    ref = np.array([mp_j0(mpmath.mpf(float(z))) for z in zs])
    assert np.max(np.abs(got - ref)) < 2.5e-16


def test_j0_exact_phase_large_arguments():
    """z = pi*I/D + delta at DHT-sized integers (N = 2^20): the phase must be
    reduced exactly, so the error stays at the rounding level although
    z ~ 3e6 (a naive cos(z - pi/4) loses ~1e-10 there)."""
    rng = np.random.default_rng(2)
    N = 2 ** 20
    D = 4 * (4 * N + 3)
    worst = 0.0
    for _ in range(60):
        k, n = (int(x) for x in rng.integers(1, N + 1, 2))
        I = (4 * k - 1) * (4 * n - 1)
        delta = float(rng.uniform(-1e-3, 1e-3))
        z = mpmath.pi * I / D + mpmath.mpf(delta)
        worst = max(worst, abs(oracle.j0_phase(I, D, delta, 0.0) - mp_j0(z)))
    assert worst < 2e-16


def test_wronskian():
    """J_1 Y_0 - J_0 Y_1 = 2/(pi z) (DLMF 10.5.2), across the series/asymptotic switch."""
    for z in np.concatenate([np.linspace(0.05, 19.9, 80), np.linspace(20.0, 300.0, 60)]):
        w = oracle.j1(z)[0] * oracle.y0(z)[0] - oracle.j0(z)[0] * oracle.y1(z)[0]
        assert abs(w * math.pi * z / 2 - 1.0) < 2e-15, z


def test_hankel_remainder_claim_sec31():
    """Sec. 3.1: with M = 10, |R_{0,10}(z)| <= 1e-15 for every z > 17.8."""
    for z in np.linspace(17.81, 50.0, 400):
        assert abs(oracle.hankel_j0(z, 10) - oracle.j0(z)[0]) <= 1e-15, z
    # and the expansion is genuinely worse below the threshold (Fig. 1)
    assert abs(oracle.hankel_j0(8.0, 10) - oracle.j0(8.0)[0]) > 1e-12


def test_roots_against_mpmath_and_lemma32():
    nmax = 2 ** 20 + 1
    b = oracle.root_offsets(nmax)
    n = np.arange(1, nmax + 1, dtype=np.float64)
    # Lemma 3.2: 0 <= b_n <= 1/(8 (n - 1/4) pi)
    assert np.all(b >= 0.0)
    assert np.all(b <= 1.0 / (8.0 * (n - 0.25) * np.pi) * (1 + 1e-14))
    j = (n - 0.25) * np.pi + b
    assert np.all(np.diff(j) > 0)
    rng = np.random.default_rng(3)
    idx = np.concatenate([np.arange(1, 41), rng.integers(41, nmax + 1, 40), [nmax]])
    for i in idx:
        ref = mpmath.besseljzero(0, int(i))
        bref = float(ref - (mpmath.mpf(int(i)) - mpmath.mpf(1) / 4) * mpmath.pi)
        assert abs(b[i - 1] - bref) <= 1e-17 + 1e-14 * abs(bref), i
    # printed by mpmath: j_{0,2..5}
    np.testing.assert_allclose(j[1:5], [5.5200781102863106, 8.6537279129110122,
                                        11.791534439014282, 14.930917708487786], rtol=0, atol=2e-15)


def _mp_grid(task, N):
    """(r_k, w_n) in mpmath for the five grids."""
    if task in ("schlomilch", "fourier_bessel"):
        r = [mpmath.mpf(k - 1) / (N - 1) for k in range(1, N + 1)]
    elif task in ("schlomilch_paper_grid", "fourier_bessel_paper_grid"):
        r = [mpmath.mpf(k) / N for k in range(1, N + 1)]
    else:
        jN = mpmath.besseljzero(0, N + 1)
        r = [mpmath.besseljzero(0, k) / jN for k in range(1, N + 1)]
    if task.startswith("schlomilch"):
        w = [mpmath.pi * n for n in range(1, N + 1)]
    else:
        w = [mpmath.besseljzero(0, n) for n in range(1, N + 1)]
    return r, w


@pytest.mark.parametrize("task", list(oracle.TASKS))
@pytest.mark.parametrize("N", [2, 13])
def test_bruteforce_sum_against_mpmath(task, N):
    rng = np.random.default_rng(10 + N)
    c = rng.standard_normal(N)
    r, w = _mp_grid(task, N)
    ref = np.array([float(mpmath.fsum(mpmath.mpf(float(c[n])) * mpmath.besselj(0, r[k] * w[n])
                                      for n in range(N))) for k in range(N)])
    got = oracle.eval_rows(task, c)
    assert np.max(np.abs(got - ref)) <= 4e-16 * np.sum(np.abs(c))


@pytest.mark.parametrize("task,N", [("dht0", 2 ** 20), ("fourier_bessel", 2 ** 16),
                                    ("schlomilch", 4096), ("dht0", 5000)])
def test_single_entries_at_full_size(task, N):
    """One matrix entry J_0(r_k w_n) at a time, against mpmath at 40 digits."""
    rng = np.random.default_rng(4)
    jN = mpmath.besseljzero(0, N + 1)
    pairs = [(1, 1), (1, N), (N, 1), (N, N), (2, N - 1), (37, 12345 % N + 1)]
    pairs += [tuple(int(x) for x in rng.integers(1, N + 1, 2)) for _ in range(20)]
    for k, n in pairs:
        if task == "dht0":
            z = mpmath.besseljzero(0, k) * mpmath.besseljzero(0, n) / jN
        elif task == "fourier_bessel":
            z = mpmath.mpf(k - 1) / (N - 1) * mpmath.besseljzero(0, n)
        else:
            z = mpmath.mpf(k - 1) / (N - 1) * n * mpmath.pi
        assert abs(oracle.entry(task, N, k, n) - mp_j0(z)) < 2.5e-16, (k, n)


def test_first_row_is_sum_of_coefficients():
    """r_1 = 0 on the (k-1)/(N-1) grid, so f_1 = sum_n c_n J_0(0) = sum_n c_n."""
    rng = np.random.default_rng(5)
    c = rng.uniform(-1, 1, 300)
    for task in ("schlomilch", "fourier_bessel"):
        f1 = oracle.eval_rows(task, c, rows=[1])[0]
        assert abs(f1 - math.fsum(c)) < 1e-13


def test_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.eval_rows("schlomilch", np.ones(1))
    with pytest.raises(ValueError):
        oracle.eval_rows("dht0", np.ones(4), rows=[5])


def test_dht_weights_against_mpmath():
    """v_n = 2/J_1(j_{0,n})^2 (Sec. 6, eq. (selfinverse)) against mpmath's own
    zeros and J_1 at 50-digit precision, on both sides of the series/Hankel
    switch at z = 20 and for a large root."""
    N = 40
    v = oracle.dht_weights(N)
    mpmath.mp.dps = 50
    for n in list(range(1, 13)) + [25, 40]:
        ref = 2 / mpmath.besselj(1, mpmath.besseljzero(0, n)) ** 2
        assert abs(v[n - 1] / float(ref) - 1) < 4e-15, n
    big = oracle.dht_weights(5000)[-1]
    ref = 2 / mpmath.besselj(1, mpmath.besseljzero(0, 5000)) ** 2
    assert abs(big / float(ref) - 1) < 1e-14


@pytest.mark.parametrize("N,bound", [(25, 2e-7), (100, 1e-9), (400, 5e-11)])
def test_dht_self_inverse(N, bound):
    """Eq. (selfinverse): (1/j_{0,N+1}^2) J D_v J D_v -> I.  With the oracle's
    forward sums and its inverse, both compositions return Gaussian c to an
    error that falls quickly with N (measured about 9e-8, 3e-10 and 9e-12; any
    dropped factor, a wrong power of J_1 or of j_{0,N+1}, or j_{0,N} in place of
    j_{0,N+1} gives errors of order 1e-2 or more)."""
    c = np.random.default_rng(N).standard_normal(N)
    back = oracle.dht0_inverse_rows(oracle.eval_rows("dht0", c))
    assert np.max(np.abs(back - c)) < bound
    again = oracle.eval_rows("dht0", oracle.dht0_inverse_rows(c))  # eq. (inverseTest)
    assert np.max(np.abs(again - c)) < bound


def test_dht_inverse_rows_subset():
    """Selected rows equal the same rows of the full inverse."""
    f = np.random.default_rng(3).standard_normal(300)
    full = oracle.dht0_inverse_rows(f)
    rows = np.array([1, 2, 150, 299, 300])
    assert np.array_equal(oracle.dht0_inverse_rows(f, rows=rows), full[rows - 1])


@pytest.mark.parametrize("nu", [1, 2, 3, 5, 8])
def test_jn_against_mpmath(nu):
    """J_nu (Schlomilch of order nu, Sec. 4) against mpmath at 40 digits: dense
    on [0, 60], on both sides of the series/Hankel switch at z = 20 + nu/2,
    and at large arguments."""
    mpmath.mp.dps = 40
    zs = list(np.linspace(0.0, 60.0, 601)) + [20 + nu / 2 - 1e-9, 20 + nu / 2 + 1e-9, 347.25, 98765.4]
    worst = max(abs(oracle.jn(nu, z)[0] - float(mpmath.besselj(nu, z))) for z in zs)
    assert worst < 1.5e-16


def test_jn_order_zero_matches_j0():
    z = np.linspace(0.0, 80.0, 801)
    assert np.array_equal(oracle.jn(0, z), oracle.j0(z))


@pytest.mark.parametrize("task", ["schlomilch", "schlomilch_paper_grid"])
@pytest.mark.parametrize("nu,shift", [(1, 0), (2, 2), (5, 0), (8, 8), (0, 3)])
def test_bruteforce_order_nu_against_mpmath(task, nu, shift):
    """f_k = sum_n c_n J_nu(r_k (n + shift) pi) (Sec. 4, Remark 4.1) at N = 2
    and 13 against mpmath sums."""
    mpmath.mp.dps = 40
    for N in (2, 13):
        c = np.random.default_rng(100 * nu + shift + N).standard_normal(N)
        ref = []
        for k in range(1, N + 1):
            r = mpmath.mpf(k - 1) / (N - 1) if task == "schlomilch" else mpmath.mpf(k) / N
            ref.append(float(mpmath.fsum(mpmath.mpf(float(c[n - 1])) * mpmath.besselj(nu, r * (n + shift) * mpmath.pi)
                                         for n in range(1, N + 1))))
        got = oracle.eval_rows(task, c, nu=nu, shift=shift)
        assert np.max(np.abs(got - np.array(ref))) <= 4e-16 * np.sum(np.abs(c))


def test_order_nu_exact_phase_at_full_size():
    """Single order-nu entries at N = 2^20 (z up to ~3.3e6), phase reduced
    exactly, against mpmath."""
    mpmath.mp.dps = 40
    N = 1 << 20
    rng = np.random.default_rng(5)
    for nu, shift in ((3, 3), (8, 0)):
        for _ in range(20):
            k, n = (int(x) for x in rng.integers(1, N + 1, 2))
            ref = mpmath.besselj(nu, mpmath.mpf(k) * (n + shift) * mpmath.pi / N)
            assert abs(oracle.entry("schlomilch_paper_grid", N, k, n, nu=nu, shift=shift) - float(ref)) < 2e-16


@pytest.mark.parametrize("task", ["fourier_bessel", "fourier_bessel_paper_grid"])
@pytest.mark.parametrize("nu", [1, 4, 8])
def test_bruteforce_fourier_bessel_order_nu(task, nu):
    """eq. (FourierBessel): f_k = sum_n c_n J_nu(r_k j_{0,n}) (order nu at the
    roots of J_0) at N = 2 and 13 against mpmath."""
    mpmath.mp.dps = 40
    for N in (2, 13):
        c = np.random.default_rng(7 * nu + N).standard_normal(N)
        j = [mpmath.besseljzero(0, n) for n in range(1, N + 1)]
        ref = []
        for k in range(1, N + 1):
            r = mpmath.mpf(k - 1) / (N - 1) if task == "fourier_bessel" else mpmath.mpf(k) / N
            ref.append(float(mpmath.fsum(mpmath.mpf(float(c[n])) * mpmath.besselj(nu, r * j[n]) for n in range(N))))
        got = oracle.eval_rows(task, c, nu=nu)
        assert np.max(np.abs(got - np.array(ref))) <= 4e-16 * np.sum(np.abs(c))


def test_order_nu_rejected_where_undefined():
    with pytest.raises(ValueError):
        oracle.eval_rows("dht0", np.ones(4), nu=1)
    with pytest.raises(ValueError):
        oracle.eval_rows("fourier_bessel", np.ones(4), shift=1)
    with pytest.raises(ValueError):
        oracle.eval_rows("schlomilch", np.ones(4), nu=13)
