"""Lockstep execution of several Softmax jobs (hs_softmax_jobs): each job's
output ciphertexts are bit for bit those of the job run alone (every
operation acts per ciphertext; the auxiliary ciphertexts of the jobs are only
batched), and every job meets the precision bar.  Toy ring N = 2^12."""
import numpy as np
import pytest

import synthetic
from oracle import softmax as S

pytestmark = pytest.mark.gpu

TOY = dict(exp_degree=7, inv_degrees=(15, 15, 31))


@pytest.fixture(scope="module")
def ctx():
    from paper_2410_11184_amd import hs
    c = hs.Context(synthetic.preset("toy12"))
    c.keygen(123)
    return c


@pytest.mark.parametrize("variant", [0, 1])
def test_jobs_match_alone_bit_for_bit(ctx, variant):
    from paper_2410_11184_amd.softmax import encrypt_logits, decrypt_outputs
    n, M, J = 16, 8.0, 3
    L = 2 * ctx.slots // n                  # m = 2 ciphertexts per job
    xs = [synthetic.logits_uniform(L, n, M, seed=500 + j) for j in range(J)]
    cts = [encrypt_logits(ctx, x, M, seed=70 + 10 * j) for j, x in enumerate(xs)]
    assert all(len(c) == 2 for c in cts)
    together = ctx.softmax([c for cs in cts for c in cs], n, M, variant=variant, jobs=J, **TOY)
    st = ctx.softmax_stats()
    for j in range(J):
        alone = ctx.softmax(cts[j], n, M, variant=variant, **TOY)
        for a, b in zip(alone, together[2 * j:2 * j + 2]):
            assert a.level == b.level and a.scale == b.scale
            assert np.array_equal(a.export(), b.export()), "job %d differs from its run alone" % j
        y = decrypt_outputs(ctx, together[2 * j:2 * j + 2], n)
        bits = S.precision_bits(S.softmax(xs[j]), y)
        assert bits["worst"] >= 16.0, (j, bits)
    print("variant", variant, "stats", st)


def test_jobs_count_must_divide(ctx):
    from paper_2410_11184_amd import hs
    from paper_2410_11184_amd.softmax import encrypt_logits
    x = synthetic.logits_uniform(4 * ctx.slots // 16, 16, 8.0, seed=9)
    cts = encrypt_logits(ctx, x, 8.0, seed=3)
    assert len(cts) == 4
    with pytest.raises(hs.HSError) as e:
        ctx.softmax(cts, 16, 8.0, jobs=3, **TOY)
    assert e.value.name == "HS_E_ARG"
