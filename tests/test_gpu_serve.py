"""Serving loop on the GPU (toy ring N = 2^12): a mix of requests of several
dimensions and sizes, two workers with their own streams; every result is bit
for bit the result of the same request served alone, and meets the precision
bar.  Continuous batching must actually have batched and overlapped."""
import numpy as np
import pytest

import synthetic
from oracle import softmax as S

pytestmark = pytest.mark.gpu

TOY = dict(exp_degree=7, inv_degrees=(15, 15, 31))


def _mix():
    rng = np.random.default_rng(77)
    reqs = []
    # dimension 16 (what the toy ring's degrees are sized for); 1..250 vectors
    # give jobs of one or two ciphertexts, i.e. two lockstep shapes
    for rid in range(10):
        V = int(rng.integers(1, 250))
        reqs.append((rid, synthetic.logits_uniform(V, 16, 8.0, seed=900 + rid)))
    reqs.append((10, synthetic.logits_uniform(5, 16, 8.0, seed=990)))
    reqs.append((11, synthetic.logits_uniform(7, 16, 8.0, seed=991)))
    return reqs


def test_results_alone_and_in_the_mix_are_identical():
    from paper_2410_11184_amd import serve
    p = synthetic.preset("toy12")
    # all requests at once: batched by shape, two workers in parallel
    srv = serve.SoftmaxServer(p, workers=2, hbm_budget_gb=4.0, variant=1, softmax_kw=TOY, key_seed=5)
    mixed = [srv.submit(rid, x, 8.0) for rid, x in _mix()]
    for r in mixed:
        assert r.done.wait(120)
    srv.close()
    assert all(r.error is None for r in mixed), [r.error for r in mixed if r.error]
    assert max(r.batch_jobs for r in mixed) > 1, "no request was batched with another"
    assert len({r.worker for r in mixed}) == 2, "one worker did all the work"
    # one at a time on a fresh server
    alone_srv = serve.SoftmaxServer(p, workers=1, hbm_budget_gb=4.0, variant=1, softmax_kw=TOY, key_seed=5)
    for (rid, x), rm in zip(_mix(), mixed):
        ra = alone_srv.submit(rid, x, 8.0)
        assert ra.done.wait(120) and ra.error is None
        assert ra.batch_jobs == 1
        assert np.array_equal(ra.result, rm.result), "request %d differs alone and in the mix" % rid
        bits = S.precision_bits(S.softmax(x), rm.result)
        assert bits["worst"] >= 16.0, (rid, bits)
    alone_srv.close()
    st = serve.latency_stats(mixed)
    print("latency", st)
    assert st["p99_s"] >= st["p50_s"] > 0
