"""Host-side failure paths and the plan cache, forced from the host:

* a device allocation made to fail (HANK_TEST_FAIL_ALLOC=n fails the n-th
  allocation) returns HANK_ENOMEM at every allocation site of a plan build and
  of the workspace, leaves out untouched, and the next call succeeds;
* the plan cache limit (hank_cache_limit) frees least recently used plans,
  never those pinned by a live batch graph, and a freed plan is rebuilt with
  bitwise the same results."""
import os

import numpy as np
import pytest

import paper_1501_01652_amd as hank
from paper_1501_01652_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_allocation_failure_returns_enomem_and_writes_nothing():
    N, eps = 20011, 1e-8  # a plan with far blocks: roots, e_k, tiles, chirp spectra, work buffers
    assert hank.plan_info("dht0", N, eps, prefer_far=1)["nblocks"] >= 1
    c = dev(inputs.coefficients("gauss", N, 2101))
    ref = host(hank.transform("dht0", c, eps, prefer_far=1))
    hank.cache_clear()
    failures = 0
    try:
        for n in range(1, 40):
            os.environ["HANK_TEST_FAIL_ALLOC"] = str(n)
            hank.cache_clear()
            out = torch.full_like(c, np.nan)
            try:
                hank.transform("dht0", c, eps, out=out, prefer_far=1)
            except hank.HankError as e:
                assert e.status == 2, e  # HANK_ENOMEM
                assert np.all(np.isnan(host(out)))
                failures += 1
                continue
            # the n-th allocation came after this call: it ran normally
            assert np.array_equal(host(out), ref)
            break
    finally:
        os.environ.pop("HANK_TEST_FAIL_ALLOC", None)
    print("allocation sites that failed cleanly:", failures)
    assert failures >= 5
    out = torch.full_like(c, np.nan)
    hank.transform("dht0", c, eps, out=out, prefer_far=1)
    assert np.array_equal(host(out), ref)


def test_cache_limit_evicts_lru_and_rebuilds_identically():
    hank.cache_clear()
    sizes = [3001, 5003, 7001, 9001, 12007]
    cs = {N: dev(inputs.coefficients("gauss", N, 2200 + N)) for N in sizes}
    first = {}
    for N in sizes:
        first[N] = host(hank.transform("fourier_bessel", cs[N], 1e-10, prefer_far=1))
    full = hank.cache_bytes()
    assert full > 0
    limit = full // 3
    try:
        hank.cache_limit(limit)
        assert hank.cache_bytes() <= limit
        for rep in range(2):
            for N in sizes:
                f = host(hank.transform("fourier_bessel", cs[N], 1e-10, prefer_far=1))
                assert np.array_equal(f, first[N])
                # at most the limit, or the one plan just used if it alone is larger
                assert hank.cache_bytes() <= max(limit, full)
        # a plan pinned by a live graph survives a limit of zero
        g = hank.BatchGraph([{"task": "fourier_bessel", "c": cs[sizes[0]], "out": torch.empty_like(cs[sizes[0]]),
                              "eps": 1e-10}])
        hank.cache_limit(0)
        assert hank.cache_bytes() > 0
        g.launch()
        g.launch()
        torch.cuda.synchronize()
        g.close()
        hank.cache_limit(0)
        assert hank.cache_bytes() == 0
    finally:
        hank.cache_limit(16 << 30)
        hank.cache_clear()
