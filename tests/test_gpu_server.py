"""The continuous-batching server (hank_server_*): every completed request
gives bitwise the result it gives alone, admission control rejects without
writing, and the statistics are consistent."""
import numpy as np
import pytest

import oracle
import paper_1501_01652_amd as hank

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _trace(seed, count, window_s):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        task = ["schlomilch", "fourier_bessel", "dht0"][int(rng.integers(0, 3))]
        N = int(rng.choice([64, 300, 1000, 2500]))
        eps = float(rng.choice([1e-4, 1e-8, 1e-14]))
        c = rng.standard_normal(N)
        out.append({"task": task, "c": dev(c), "out": dev(np.full(N, np.nan)), "eps": eps,
                    "arrival": float(rng.uniform(0, window_s)), "host": c})
    return out


@pytest.mark.parametrize("max_batch", [1, 8])
def test_server_results_equal_alone(max_batch):
    reqs = _trace(31, 40, 0.05)
    with hank.Server(budget_bytes=1 << 32, max_batch=max_batch, max_pending=1000) as srv:
        tickets = [srv.submit(r, arrival_s=r["arrival"]) for r in reqs]
        srv.start()
        srv.drain()
        st = srv.stats()
        states = [srv.status(t)[0] for t in tickets]
    assert states == ["done"] * len(reqs)
    assert st["completed"] == len(reqs) and st["rejected"] == 0
    assert st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    assert st["mean_batch"] >= 1.0
    for r in reqs:
        alone = host(hank.transform(r["task"], r["c"], r["eps"]))
        assert np.array_equal(host(r["out"]), alone)
    # and the values are right
    for r in reqs[:6]:
        ref = oracle.eval_rows(r["task"], r["host"])
        assert np.max(np.abs(host(r["out"]) - ref)) <= 10 * r["eps"] * np.sum(np.abs(r["host"]))


def test_server_rejects_when_queue_full_and_writes_nothing():
    reqs = _trace(32, 30, 0.0)  # a burst: everything arrives at t = 0
    for r in reqs:
        r["arrival"] = 0.0
    with hank.Server(budget_bytes=1 << 32, max_batch=4, max_pending=3) as srv:
        tickets = [srv.submit(r, arrival_s=0.0) for r in reqs]
        srv.start()
        srv.drain()
        st = srv.stats()
        states = [srv.status(t)[0] for t in tickets]
    assert st["rejected"] > 0 and st["completed"] + st["rejected"] == len(reqs)
    for r, s in zip(reqs, states):
        out = host(r["out"])
        if s == "rejected":
            assert np.all(np.isnan(out))
        else:
            assert s == "done" and not np.any(np.isnan(out))


def test_server_rejects_requests_larger_than_the_budget():
    N = 1 << 16
    c = dev(np.random.default_rng(3).standard_normal(N))
    out = dev(np.full(N, np.nan))
    with hank.Server(budget_bytes=1 << 20, max_batch=4, max_pending=10) as srv:
        t = srv.submit({"task": "dht0", "c": c, "out": out, "eps": 1e-8}, arrival_s=0.0)
        srv.start()
        srv.drain()
        assert srv.status(t)[0] == "rejected"
    assert np.all(np.isnan(host(out)))
