"""The HIP bootstrapping (hs_bootstrap, hs_dbg_bootstrap_stage) against the
oracle's (oracle/bootstrap.py), stage by stage, on the same keys and input
ciphertexts (small bootstrapping ring, N = 2^10):

* after ModRaise the ciphertexts are equal word for word (integer steps
  only);
* every later stage decrypts to the oracle's value within 2^-30 of the
  values' size, at the same level and scale: the linear-transform plaintexts
  come from floating-point matrices computed in a different order on each
  side (dense stage products here, sparse ones there) and enter as rounded
  integers, so from CoeffToSlot on the words differ while the values agree
  to the noise level (about 2^-33 at the output's scale 2^40), far below
  the approximation error the stages share (the bootstrapping's own
  precision, about 2^-26 here);
* the Softmax schedule with bootstraps inside (N = 2^10 with 10 user
  levels) decrypts to the oracle schedule's output likewise.
"""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

SEED = 5150


@pytest.fixture(scope="module")
def pair():
    from paper_2410_11184_amd import hs
    from oracle import ckks
    from oracle.bootstrap import Bootstrapper
    p = synthetic.preset("boot10")
    g = hs.Context(p)
    o = ckks.Context(**p)
    g.keygen(SEED)
    o.keygen(SEED)
    return g, o, Bootstrapper(o, p["boot"], p["user_top"], p["log_scale"])


def _close(g, o, gct, oct_, what, tol=2.0 ** -30):
    assert gct.level == oct_.level, (what, gct.level, oct_.level)
    assert abs(gct.scale / oct_.scale - 1.0) < 1e-12, (what, gct.scale, oct_.scale)
    a = g.decrypt(gct)
    b = o.decrypt_decode(oct_)
    size = max(1.0, float(np.max(np.abs(b))))
    diff = float(np.max(np.abs(a - b)))
    print("%s: max |hip - oracle| = 2^%.1f (values up to %.3g)" % (what, np.log2(diff + 1e-300), size))
    assert diff < tol * size, what


@pytest.mark.parametrize("level", [0, 2])
def test_stages_match_the_oracle(pair, level):
    g, o, bs = pair
    r = np.random.default_rng(level)
    z = 0.9 * (r.uniform(-1, 1, o.slots) + 1j * r.uniform(-1, 1, o.slots)) / np.sqrt(2)
    gx = g.encrypt(z, level, o.delta, 77 + level)
    ox = o.encode_encrypt(z, o.delta, level, 77 + level)
    w = gx.export()
    assert np.array_equal(w[0], ox.c[0]) and np.array_equal(w[1], ox.c[1])
    tr = {}
    oy = bs.bootstrap(ox, 1.0, trace=tr)
    # ModRaise: word for word
    s1 = g.bootstrap_stage(gx, 1)
    w1 = s1.export()
    assert s1.level == tr[1].level and s1.scale == tr[1].scale
    assert np.array_equal(w1[0], tr[1].c[0]) and np.array_equal(w1[1], tr[1].c[1])
    for stage in range(2, 10):
        _close(g, o, g.bootstrap_stage(gx, stage), tr[stage], "stage %d" % stage)
    gy = g.bootstrap(gx)
    _close(g, o, gy, oy, "output")
    assert np.max(np.abs(g.decrypt(gy) - z)) < 2.0 ** -22


@pytest.mark.parametrize("variant", [0, 1, "newton", "newton-refresh"])
def test_softmax_with_bootstraps_matches_the_oracle(variant):
    from paper_2410_11184_amd import hs
    from oracle import ckks, schedule, softmax as S
    from oracle.bootstrap import Bootstrapper
    p = synthetic.preset("boot10u")
    g = hs.Context(p)
    o = ckks.Context(**p)
    g.keygen(SEED + 1)
    o.keygen(SEED + 1)
    bs = Bootstrapper(o, p["boot"], p["user_top"], p["log_scale"])
    # "newton": Algorithm SM at n = 32, M = 32, degree-15 first guesses and one
    # Newton step per inverse square root, bootstraps between; "newton-refresh":
    # degree-31 guesses, whose depth plus the step's levels exceed the 10
    # levels a bootstrapping restores, so each guess is bootstrapped itself
    # before its Newton step
    nw = str(variant).startswith("newton")
    kw = dict(inv_degrees=(31, 31, 31) if variant == "newton-refresh" else (15, 15, 15), newton_steps=1) if nw else {}
    n, M, m = (32, 32.0, 1) if nw else (16, 8.0, 1)
    seed_off = {"newton": 2, "newton-refresh": 3}.get(variant, variant)
    variant = 0 if nw else variant
    L = m * o.slots // n
    x = synthetic.logits_uniform(L, n, M, seed=61 + seed_off)
    packed = S.pack(x, m, o.slots)
    scale = o.delta * 2.0 / M
    gx = [g.encrypt(packed[0], p["user_top"], scale, 90)]
    ox = [o.encode_encrypt(packed[0], scale, p["user_top"], 90)]
    gy = g.softmax(gx, n, M, variant=variant, **kw)
    gst = g.softmax_stats()
    st = {}
    oy = schedule.softmax(o, ox, n, M, variant=variant,
                          bootstrap=lambda c, bound, mask_L: bs.bootstrap(c, bound, mask_L), stats=st,
                          boot_top=p["user_top"], **kw)
    assert gst["bootstraps"] == st["bootstraps"] > 0, (gst, st)
    _close(g, o, gy[0], oy[0], "softmax output", tol=2.0 ** -24)
    y = S.unpack(np.stack([g.decrypt(gy[0]).real]), n)
    assert S.precision_bits(S.softmax(x), y)["worst"] >= 16.0
