"""The batched workload at its full sizes (N log-uniform up to 2^16, up to 64
right-hand sides, the three tasks and eps values): a batch of 40 of its
requests -- the largest ones included -- gives bitwise the results of the
same requests one call at a time, and sampled right-hand sides match the
oracle on sampled rows within 10 eps sum|c|."""
import numpy as np
import pytest

import oracle
import paper_1501_01652_amd as hank
from paper_1501_01652_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _requests(count=40):
    specs = inputs.batch_specs(1024)
    by_size = sorted(range(len(specs)), key=lambda i: specs[i]["N"] * specs[i]["nrhs"])
    pick = sorted(set(by_size[::len(specs) // (count - 4)] + by_size[-4:]))
    reqs = []
    for i in pick:
        sp = specs[i]
        rng = np.random.default_rng(sp["seed"])
        c = rng.uniform(-1.0, 1.0, (sp["nrhs"], sp["N"]))
        if sp["nrhs"] == 1:
            c = c[0]
        cd = torch.from_numpy(c).to("cuda")
        reqs.append({"task": sp["task"], "c": cd, "out": torch.full_like(cd, np.nan), "eps": sp["eps"], "host": c})
    return reqs


def test_batch_at_full_sizes_equals_single_calls_and_oracle():
    reqs = _requests()
    assert max(r["c"].shape[-1] for r in reqs) >= 1 << 15
    assert max(r["c"].shape[0] if r["c"].dim() > 1 else 1 for r in reqs) >= 48
    hank.batch(reqs)
    torch.cuda.synchronize()
    for r in reqs:
        alone = host(hank.transform(r["task"], r["c"], r["eps"]))
        assert np.array_equal(host(r["out"]), alone)
    # the largest requests against the oracle: first and last right-hand side
    big = sorted(reqs, key=lambda r: r["c"].numel())[-6:]
    for r in big:
        f = host(r["out"])
        c = r["host"]
        N = c.shape[-1]
        rows = inputs.sampled_rows(N, 12, seed=inputs.SEED_SAMPLED_ROWS)
        cols = [0, c.shape[0] - 1] if c.ndim == 2 else [None]
        for j in cols:
            cj, fj = (c, f) if j is None else (c[j], f[j])
            ref = oracle.eval_rows(r["task"], cj, rows=rows)
            err = float(np.max(np.abs(fj[rows - 1] - ref)))
            tol = 10.0 * r["eps"] * float(np.sum(np.abs(cj)))
            print("%s N=%d eps=%g rhs %s: max err %.3e (C = %.3g)" % (r["task"], N, r["eps"], j, err,
                                                                       err / (tol / 10.0)))
            assert err <= tol
