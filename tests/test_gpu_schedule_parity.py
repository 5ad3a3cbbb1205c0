"""The whole encrypted Softmax schedule (hs_softmax: Algorithm SM and SM
version B with the auxiliary thread and the many-ciphertext packing) against
the oracle's schedule (oracle/schedule.py, oracle/polyeval.py) on the same
keys and encryptions: the output ciphertexts must be equal word for word.

Both sides take every floating-point decision (polynomial coefficients,
intervals, scales, integer constants) by the same specification, so one
differing word would show a schedule, a polynomial or an evaluation-order
mismatch.  The intermediate y0 = exp(x / 2^k) / sqrt(n) (after the first
polynomial) is compared first, to localise a difference.  Toy ring N = 2^12
(no bootstrapping: the schedule must fit its 23 levels)."""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

SEED = 4242
CASES = [
    # (variant, m, n, M, k (0: the Theorem's), exp degree, normalisation
    # degrees, worst-case bits these degrees reach on this ring)
    (0, 1, 16, 8.0, 0, 7, (15, 15, 31), 16.0),
    (1, 1, 16, 8.0, 0, 7, (15, 15, 31), 16.0),
    (1, 2, 16, 8.0, 0, 7, (15, 15, 31), 16.0),
    # four ciphertexts, four rotate-and-add steps: the toy ring's 23 levels
    # hold n = 64 only with low degrees (the Theorem's k = 1 leaves the single
    # normalisation on [e^-8, 1]; k = 2 ends at level 2), so the precision bar
    # here is that of these degrees; n = 64 reaches 16 bits with
    # bootstrapping at N = 2^16
    (1, 4, 64, 8.0, 2, 7, (15, 15, 31), 10.0),
]
# (variant, m, n, M, k, exp degree, normalisation degrees, bits, power):
# normalize-and-cube (the appendix on other normalisations; k = 1 from
# M / 3^k ~ ln n), and dimensions that are not powers of two (12 packed as 16,
# the 4 extra coordinates masked after the exponential)
# then (Newton steps, mask mode): the inverse square roots refined by one
# Newton step from degree-7 first guesses (Appendix A), with the indicator
# mask folded into that step or with the averaging mask (the toy ring's
# levels allow no more: about 8 bits, 3.4 without the Newton step), version
# B with the averaging mask, and version B with a Newton step in its last
# iteration
MORE = [
    (0, 1, 8, 4.0, 0, 7, (31, 31, 31), 14.0, 3, 0, 0),
    (1, 2, 12, 8.0, 0, 7, (15, 15, 31), 16.0, 2, 0, 0),
    (0, 1, 12, 8.0, 0, 7, (15, 15, 15), 13.0, 2, 0, 0),
    (0, 1, 16, 8.0, 0, 7, (7, 7, 7), 8.0, 2, 1, 0),
    (0, 2, 16, 8.0, 0, 7, (7, 7, 7), 8.0, 2, 1, 1),
    (1, 2, 16, 8.0, 0, 7, (15, 15, 31), 16.0, 2, 0, 1),
    # version B with one Newton step in its last iteration (its only inverse
    # square root), from a degree-7 first guess
    (1, 2, 16, 8.0, 0, 7, (15, 15, 7), 8.0, 2, 1, 0),
]


def _case_id(c):
    c = c + (2, 0, 0)[len(c) - 8:]
    return "v%d-m%d-n%d-t%d-nw%d-avg%d" % (c[0], c[1], c[2], c[8], c[9], c[10])


@pytest.fixture(scope="module")
def pair():
    from paper_2410_11184_amd import hs
    from oracle import ckks
    p = synthetic.preset("toy12")
    g = hs.Context(p)
    o = ckks.Context(**p)
    g.keygen(SEED)
    o.keygen(SEED)
    return g, o


def _inputs(g, o, n, M, m, seed, headroom=False):
    from oracle import softmax as S
    L = m * o.slots // S.padded(n)
    x = synthetic.logits_uniform(L, n, M, seed=seed)
    packed = S.pack(x, m, o.slots)
    scale = o.delta * 2.0 / M
    top = synthetic.preset("toy12")["user_top"]
    if headroom:
        scale *= float(o.q[top])
    gx = [g.encrypt(packed[j], top, scale, seed + 100 + j) for j in range(m)]
    ox = [o.encode_encrypt(packed[j], scale, top, seed + 100 + j) for j in range(m)]
    for a, b in zip(gx, ox):
        w = a.export()
        assert np.array_equal(w[0], b.c[0]) and np.array_equal(w[1], b.c[1])
    return x, gx, ox


def _compare(g, o, gy, oy, what):
    assert len(gy) == len(oy)
    for i, (a, b) in enumerate(zip(gy, oy)):
        assert a.level == b.level, (what, i, a.level, b.level)
        assert a.scale == b.scale, (what, i, a.scale, b.scale)
        w = a.export()
        for k in range(2):
            if not np.array_equal(w[k], b.c[k]):
                diff = np.max(np.abs(g.decrypt(a) - o.decrypt_decode(b)))
                bad = np.argwhere(w[k] != b.c[k])
                pytest.fail("%s: ciphertext %d component %d differs in %d words (first %s); "
                            "decrypted max difference %.3g" % (what, i, k, len(bad), bad[0], diff))


@pytest.mark.parametrize("case", CASES + MORE, ids=_case_id)
def test_schedule_matches_oracle(pair, case):
    from oracle import schedule, softmax as S
    g, o = pair
    variant, m, n, M, k, dexp, dinv, want_bits, t, nw, mm = case + (2, 0, 0)[len(case) - 8:]
    opt = dict(power=t, newton_steps=nw, mask_mode=mm)
    x, gx, ox = _inputs(g, o, n, M, m, seed=700 + 10 * variant + m)
    # first polynomial alone
    gy0 = g.softmax(gx, n, M, variant=variant, k=k, exp_degree=dexp, inv_degrees=dinv, debug_stop=0, **opt)
    oy0 = schedule.softmax(o, ox, n, M, variant=variant, k=k, exp_degree=dexp, inv_degrees=dinv, debug_stop=0,
                           **opt)
    _compare(g, o, gy0, oy0, "y0")
    # the whole schedule
    gy = g.softmax(gx, n, M, variant=variant, k=k, exp_degree=dexp, inv_degrees=dinv, **opt)
    oy = schedule.softmax(o, ox, n, M, variant=variant, k=k, exp_degree=dexp, inv_degrees=dinv, **opt)
    _compare(g, o, gy, oy, "output")
    y = S.unpack(np.stack([o.decrypt_decode(c).real for c in oy]), n)
    bits = S.precision_bits(S.softmax(x), y)
    print(case, bits)
    assert bits["worst"] >= want_bits


@pytest.mark.parametrize("variant", [0, 1])
def test_input_one_rescale_above_matches_oracle(pair, variant):
    # inputs at scale (2 Delta / M) q_l: the schedule starts with one rescale
    # (the encryption noise divided by q_l) instead of the declared-scale change
    from oracle import schedule, softmax as S
    g, o = pair
    n, M, m = 16, 8.0, 2
    x, gx, ox = _inputs(g, o, n, M, m, seed=760 + variant, headroom=True)
    kw = dict(variant=variant, exp_degree=7, inv_degrees=(15, 15, 31))
    gy0 = g.softmax(gx, n, M, debug_stop=0, **kw)
    oy0 = schedule.softmax(o, ox, n, M, debug_stop=0, **kw)
    _compare(g, o, gy0, oy0, "y0")
    assert gy0[0].level == gx[0].level - 1 - 4           # one rescale, then the degree-7 polynomial
    gy = g.softmax(gx, n, M, **kw)
    oy = schedule.softmax(o, ox, n, M, **kw)
    _compare(g, o, gy, oy, "output")
    y = S.unpack(np.stack([o.decrypt_decode(c).real for c in oy]), n)
    assert S.precision_bits(S.softmax(x), y)["worst"] >= 16.0


@pytest.mark.parametrize("variant", [0, 1])
def test_interpolated_normalisation_matches_oracle(pair, variant):
    # approx = 1: Chebyshev interpolants instead of the weighted minimax
    # approximants for the normalisation polynomials
    from oracle import schedule, softmax as S
    g, o = pair
    n, M, m = 16, 8.0, 2
    x, gx, ox = _inputs(g, o, n, M, m, seed=780 + variant)
    kw = dict(variant=variant, exp_degree=7, inv_degrees=(15, 15, 31), approx=1)
    gy = g.softmax(gx, n, M, **kw)
    oy = schedule.softmax(o, ox, n, M, **kw)
    _compare(g, o, gy, oy, "output")
    y = S.unpack(np.stack([o.decrypt_decode(c).real for c in oy]), n)
    assert S.precision_bits(S.softmax(x), y)["worst"] >= 16.0


@pytest.mark.parametrize("case", [(16, 4.0, 2, 2, (31, 31, 31), 13.5), (16, 8.0, 2, 2, (7, 7, 15), 7.0),
                                  (16, 8.0, 1, 4, (7, 7, 15), 7.0), (16, 8.0, 4, 8, (7, 7, 15), 7.0)],
                         ids=["k1-m2-J2", "k2-m2-J2", "k2-m1-J4", "k2-m4-J8-two-packed"])
def test_packed_jobs_match_oracle(pair, case):
    # version B with the jobs' auxiliary ciphertexts packed (hs_softmax_jobs,
    # merge = 1; n / m jobs per auxiliary ciphertext, so 8 jobs of m = 4 take
    # two) against the oracle's packed schedule, word for word; k = 2 takes
    # the packed Lambda through a version-B step (the
    # toy ring's 23 levels hold it only with low degrees, so the precision
    # bar is that of these degrees); each job's logits differ
    from oracle import schedule, softmax as S
    g, o = pair
    n, M, m, J, dinv, want_bits = case
    xs, gxs, oxs = [], [], []
    for jb in range(J):
        x, gx, ox = _inputs(g, o, n, M, m, seed=800 + 10 * jb + m)
        xs.append(x)
        gxs += gx
        oxs += ox
    kw = dict(variant=1, exp_degree=7, inv_degrees=dinv)
    gy = g.softmax(gxs, n, M, jobs=J, merge=1, **kw)
    oy = schedule.softmax(o, oxs, n, M, jobs=J, merge=True, **kw)
    _compare(g, o, gy, oy, "output")
    for jb in range(J):
        y = S.unpack(np.stack([o.decrypt_decode(c).real for c in oy[jb * m:(jb + 1) * m]]), n)
        bits = S.precision_bits(S.softmax(xs[jb]), y)
        print(case, jb, bits)
        assert bits["worst"] >= want_bits, (jb, bits)


def test_packed_jobs_refusals(pair):
    from paper_2410_11184_amd import hs
    g, o = pair
    n, M, m = 16, 8.0, 2
    _, gx, _ = _inputs(g, o, n, M, m, seed=890)
    for kw in (dict(variant=0), dict(variant=1, mask_mode=1), dict(variant=1, newton_steps=1)):
        with pytest.raises(hs.HSError) as e:
            g.softmax(gx, n, M, jobs=2, merge=1, exp_degree=7, inv_degrees=(7, 7, 15), **kw)
        assert e.value.name == "HS_E_PARAM", kw
    # more jobs than blocks of L slots and not a multiple of them: n / m = 8
    # blocks, 12 jobs of m = 2
    cts = [gx[i % m] for i in range(24)]
    with pytest.raises(hs.HSError) as e:
        g.softmax(cts, n, M, jobs=12, merge=1, variant=1, exp_degree=7, inv_degrees=(7, 7, 15))
    assert e.value.name == "HS_E_PARAM"
