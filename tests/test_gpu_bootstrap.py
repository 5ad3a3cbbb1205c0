"""Bootstrapping: dec(BTS(ct)) ~ dec(ct) (the defining property; Section
2.2, "Levels").  The pipeline is composite, so its check is the decrypted
precision, on the small ring N = 2^10 with the same level structure as the
N = 2^16 parameters."""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2410_11184_amd import hs
    c = hs.Context(synthetic.preset("boot10"))
    c.keygen(4242)
    return c


def _bits(err):
    return -np.log2(max(err, 2.0 ** -60))


@pytest.mark.parametrize("level,cplx", [(0, False), (3, False), (0, True)])
def test_bootstrap_precision(ctx, level, cplx):
    r = np.random.default_rng(level + 10 * cplx)
    z = r.uniform(-1, 1, ctx.slots)
    if cplx:
        z = z + 1j * r.uniform(-1, 1, ctx.slots)
    ct = ctx.encrypt(z, level, ctx.delta, 17)
    out = ctx.bootstrap(ct)
    assert out.level == ctx.user_top
    got = ctx.decrypt(out)
    err = np.max(np.abs(got - z))
    print("level", level, "complex", cplx, "bootstrap precision bits", _bits(err))
    assert _bits(err) >= 18.0
    # the refreshed ciphertext computes: square it at the top user level
    sq = ctx.decrypt(ctx.mult(out, out))
    assert np.max(np.abs(sq - z * z)) < 2 ** -16


def test_bootstrap_small_values_keep_absolute_precision(ctx):
    z = np.random.default_rng(5).uniform(0, 1.0 / 256, ctx.slots)
    out = ctx.bootstrap(ctx.encrypt(z, 1, ctx.delta, 3))
    assert np.max(np.abs(ctx.decrypt(out).real - z)) < 2 ** -18
