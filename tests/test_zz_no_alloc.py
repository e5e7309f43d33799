"""The allocation-free entry point hank_transform_noalloc (through the C ABI)
against hank_transform on the same inputs: two calls in a row, the second with
a smaller input, each within the parity bar eps * sum|c| of the ordinary
entry point's result (and of the oracle on sampled rows); and its two error
paths (no cached plan; a workspace larger than the static scratch), which
leave out untouched."""
import numpy as np
import pytest

import oracle
import paper_1501_01652_amd as hank
from paper_1501_01652_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
C_TOL = 10.0


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def _check_pair(task, N, eps, nrhs, seed, **kw):
    c = inputs.coefficients("gauss", N * nrhs, seed).reshape((nrhs, N) if nrhs > 1 else (N,))
    cd = _dev(c)
    ref = hank.transform(task, cd, eps, **kw)  # builds and caches the plan
    torch.cuda.synchronize()
    cache_before = hank.cache_bytes()
    out = torch.full_like(cd, np.nan)
    hank.transform_noalloc(task, cd, eps, out, **kw)
    torch.cuda.synchronize()
    assert hank.cache_bytes() == cache_before  # no plan built
    f, r = out.cpu().numpy(), ref.cpu().numpy()
    assert np.all(np.isfinite(f))
    for j in range(nrhs):
        cj = c[j] if nrhs > 1 else c
        fj, rj = (f[j], r[j]) if nrhs > 1 else (f, r)
        l1 = float(np.sum(np.abs(cj)))
        d = float(np.max(np.abs(fj - rj)))
        print("noalloc %s N=%d eps=%g rhs %d: max|noalloc - transform| = %.3e (%.2e eps sum|c|)"
              % (task, N, eps, j, d, d / (eps * l1)))
        assert d <= eps * l1
        rows = inputs.sampled_rows(N, 24, seed=inputs.SEED_SAMPLED_ROWS + j)
        o = oracle.eval_rows(task, cj, rows=rows)
        e = float(np.max(np.abs(fj[rows - 1] - o)))
        assert e <= C_TOL * eps * l1, (e, C_TOL * eps * l1)


def test_noalloc_two_calls_second_smaller():
    # the first call: a DHT whose plan has far-field blocks (FP64 transforms);
    # the second: a smaller Fourier-Bessel transform of three right-hand sides
    assert hank.plan_info("dht0", 1 << 17, 1e-8, precision=1)["nblocks"] >= 1
    _check_pair("dht0", 1 << 17, 1e-8, 1, 1701, precision=1)
    assert hank.plan_info("fourier_bessel", 3000, 1e-14, prefer_far=1, nrhs=3)["nblocks"] >= 1
    _check_pair("fourier_bessel", 3000, 1e-14, 3, 1702, prefer_far=1)


def test_noalloc_errors_leave_out_untouched():
    N = 4099
    cd = _dev(inputs.coefficients("gauss", N, 1703))
    out = torch.full_like(cd, 7.0)
    # no cached plan for these arguments: nothing is built or written
    hank.cache_clear()
    with pytest.raises(hank.HankError) as ei:
        hank.transform_noalloc("schlomilch", cd, 3e-9, out)
    assert ei.value.status == 4 and "cached" in str(ei.value)
    # a workspace beyond the static scratch: 64 right-hand sides at N = 2^20
    # need 2^21-point FFT buffers of 2 GiB for a single group
    N2, nrhs = 1 << 20, 64
    c2 = torch.randn((nrhs, N2), dtype=torch.float64, device="cuda", generator=torch.Generator(
        device="cuda").manual_seed(1704))
    hank.transform("dht0", c2, 1e-8)  # caches the plan
    o2 = torch.full_like(c2, 7.0)
    with pytest.raises(hank.HankError) as ei:
        hank.transform_noalloc("dht0", c2, 1e-8, o2)
    assert ei.value.status == 4 and "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0)) and bool(torch.all(o2 == 7.0))
    del c2, o2
    hank.cache_clear()
