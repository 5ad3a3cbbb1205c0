"""Captured Softmax schedules (hs_softmax_plan_*): the schedule of
hs_softmax_jobs recorded once as a HIP graph and replayed on new inputs.

Each plan is replayed several times on different inputs, with eager work
(the same call through hs_softmax_jobs) and synchronisations between the
replays, and every replay must equal the eager result bit for bit.  Toy ring
N = 2^12 (no bootstrapping) and the bootstrapping ring N = 2^10 (the main and
auxiliary ciphertexts are refreshed inside the captured schedule, 10 user
levels)."""
import numpy as np
import pytest

import synthetic
from oracle import softmax as S

pytestmark = pytest.mark.gpu

TOY = dict(exp_degree=7, inv_degrees=(15, 15, 31))


@pytest.fixture(scope="module")
def toy():
    from paper_2410_11184_amd import hs
    c = hs.Context(synthetic.preset("toy12"))
    c.keygen(321)
    return c


@pytest.fixture(scope="module")
def boot():
    from paper_2410_11184_amd import hs
    c = hs.Context(synthetic.preset("boot10u"))
    c.keygen(654)
    return c


def _replays(ctx, n, M, m, jobs, variant, kw, seeds):
    from paper_2410_11184_amd.softmax import encrypt_logits, decrypt_outputs
    L = m * ctx.slots // n
    xs = [synthetic.logits_uniform(L, n, M, seed=s) for s in seeds]
    first = encrypt_logits(ctx, xs[0], M, seed=seeds[0] + 7)
    assert len(first) == m
    plan = ctx.softmax_plan(first, n, M, variant=variant, jobs=jobs, **kw)
    nodes, arena = plan.info()
    assert nodes > 0 and arena > 0
    for r, x in enumerate(xs):
        cts = encrypt_logits(ctx, x, M, seed=seeds[r] + 7)
        g = plan.run(cts)
        st_g = ctx.softmax_stats()
        e = ctx.softmax(cts, n, M, variant=variant, jobs=jobs, **kw)
        st_e = ctx.softmax_stats()
        assert (st_g["k"], st_g["bootstraps"]) == (st_e["k"], st_e["bootstraps"])
        for a, b in zip(e, g):
            assert a.level == b.level and a.scale == b.scale
            assert np.array_equal(a.export(), b.export()), "replay %d differs from the eager call" % r
        ctx.sync()
    y = decrypt_outputs(ctx, g, n)
    plan.close()
    return xs[-1], y, nodes


@pytest.mark.parametrize("variant", [0, 1])
def test_toy_plan_replays_match_eager(toy, variant):
    x, y, nodes = _replays(toy, 16, 8.0, 2, 1, variant, TOY, [900, 901, 902])
    bits = S.precision_bits(S.softmax(x), y)
    print("toy variant", variant, "nodes", nodes, bits)
    assert bits["worst"] >= 16.0


def test_toy_plan_jobs(toy):
    # 2 jobs of 2 ciphertexts in lockstep
    _replays(toy, 16, 8.0, 4, 2, 1, TOY, [910, 911])


@pytest.mark.parametrize("variant", [0, 1])
def test_bootstrapping_plan_replays_match_eager(boot, variant):
    _, _, nodes = _replays(boot, 16, 8.0, 1, 1, variant, {}, [920, 921, 922])
    assert boot.softmax_stats()["bootstraps"] > 0
    print("boot10u variant", variant, "nodes", nodes)


def test_packed_jobs_plan_replays_match_eager(boot):
    # two version-B jobs with their auxiliary ciphertexts packed into one,
    # bootstrapped inside the captured schedule (degrees 15 / 15 / 31: the
    # packing's extra level in the last step leaves the default degree-127
    # polynomial more levels than the ring's 10 user levels)
    _, _, nodes = _replays(boot, 16, 8.0, 2, 2, 1, dict(merge=1, **TOY), [940, 941, 942])
    assert boot.softmax_stats()["bootstraps"] > 0
    print("boot10u packed jobs, nodes", nodes)


def test_plan_rejects_other_shapes(toy):
    from paper_2410_11184_amd import hs
    from paper_2410_11184_amd.softmax import encrypt_logits
    x = synthetic.logits_uniform(2 * toy.slots // 16, 16, 8.0, seed=930)
    cts = encrypt_logits(toy, x, 8.0, seed=1)
    plan = toy.softmax_plan(cts, 16, 8.0, variant=1, **TOY)
    low = [toy.encrypt(np.zeros(toy.slots), toy.user_top - 1, toy.delta * 2.0 / 8.0, 5 + i) for i in range(2)]
    with pytest.raises(hs.HSError) as e:
        plan.run(low)
    assert e.value.name == "HS_E_LEVEL"
    with pytest.raises(ValueError):
        plan.run(cts[:1])
    plan.close()


def test_plan_refuses_capture_while_profiling(toy):
    # the launch profiler records events around launches: none may enter a graph
    from paper_2410_11184_amd import hs
    from paper_2410_11184_amd.softmax import encrypt_logits
    x = synthetic.logits_uniform(2 * toy.slots // 16, 16, 8.0, seed=940)
    cts = encrypt_logits(toy, x, 8.0, seed=2)
    toy.prof_enable(True)
    try:
        with pytest.raises(hs.HSError) as e:
            toy.softmax_plan(cts, 16, 8.0, variant=1, **TOY)
        assert e.value.name == "HS_E_STATE"
    finally:
        toy.prof_enable(False)
        toy.prof_collect()


def test_keygen_refused_while_a_plan_lives():
    # a plan's graph holds the device addresses of the keys it was recorded
    # with: new keys are refused until the plan is destroyed (the call is
    # refused up front, so no replay ever reads freed key memory)
    from paper_2410_11184_amd import hs
    from paper_2410_11184_amd.softmax import encrypt_logits
    c = hs.Context(synthetic.preset("toy12"))
    c.keygen(322)
    x = synthetic.logits_uniform(2 * c.slots // 16, 16, 8.0, seed=950)
    cts = encrypt_logits(c, x, 8.0, seed=3)
    plan = c.softmax_plan(cts, 16, 8.0, variant=1, **TOY)
    with pytest.raises(hs.HSError) as e:
        c.keygen(323)
    assert e.value.name == "HS_E_STATE"
    g = plan.run(cts)                       # the plan still replays on its keys
    e_out = c.softmax(cts, 16, 8.0, variant=1, **TOY)
    assert all(np.array_equal(a.export(), b.export()) for a, b in zip(e_out, g))
    plan.close()
    c.keygen(323)                           # allowed once the plan is gone
