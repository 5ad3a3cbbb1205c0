"""Pins of the Softmax oracle: the definition's special cases, the
doubling identity, the Cauchy-Schwarz bound, the exact twins of the paper's
loops, the packing, the precision theorem's bound under fixed-point noise,
and the polynomial approximations' own optimality conditions."""
import json
import math
import os

import numpy as np
import pytest

from oracle import softmax as S
from oracle import polyfit as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_softmax_special_cases():
    n = 64
    assert np.allclose(S.softmax(np.full((3, n), -7.0)), 1.0 / n, rtol=0, atol=1e-16)
    M = 30.0
    x = np.full(n, -M)
    x[5] = 0.0
    y = S.softmax(x[None])[0]
    assert abs(y[5] - 1.0 / (1.0 + (n - 1) * math.exp(-M))) < 2e-15
    a, b = -1.25, -4.0
    y = S.softmax(np.array([[a, b]]))[0]
    assert abs(y[0] - 1.0 / (1.0 + math.exp(b - a))) < 2e-15
    # shift invariance (Eq. eq:normalized_sm)
    x = np.random.default_rng(0).uniform(-9, 0, (4, 32))
    assert np.allclose(S.softmax(x), S.softmax(x - 3.5), atol=1e-15)


def test_doubling_identity_and_cauchy_schwarz():
    x = np.random.default_rng(1).uniform(-128, 0, (20, 256))
    for j in range(0, 8):
        y = S.softmax(x / 2 ** j)
        s2 = (y * y).sum(-1)
        assert np.all(s2 >= 1 / 256 - 1e-15) and np.all(s2 <= 1 + 1e-15)
        if j > 0:
            assert np.allclose(S.softmax(x / 2 ** (j - 1)), y * y / s2[:, None], atol=1e-14)


@pytest.mark.parametrize("n,M", [(16, 8.0), (256, 128.0), (128, 64.0), (1024, 256.0)])
def test_exact_twins_equal_softmax(n, M):
    x = np.random.default_rng(n).uniform(-M, 0, (8, n))
    ref = S.softmax(x)
    for k in (S.theorem_k(n, M), S.table_k(M)):
        assert np.max(np.abs(S.main_loop(x, k) - ref)) < 1e-12
        assert np.max(np.abs(S.softmax_b(x, k) - ref)) < 1e-12
        assert np.allclose(S.main_loop(x, k).sum(-1), 1.0, atol=1e-12)


def test_k_rules():
    # Theorem: k = ceil(log M - log ln n); tables: range [-2^k, 0]
    assert [S.theorem_k(n, M) for n, M in [(16, 8), (256, 128), (128, 64), (32768, 256)]] == [2, 5, 4, 5]
    assert [S.table_k(M) for M in (8, 128, 64, 256)] == [3, 7, 6, 8]


@pytest.mark.parametrize("m", [1, 4, 64])
def test_packed_twin(m):
    n, slots = 256, 1 << 12
    L = m * slots // n
    x = np.random.default_rng(m).uniform(-128, 0, (L, n))
    packed = S.pack(x, m, slots)
    assert np.array_equal(S.unpack(packed, n), x)
    for variant in ("SM", "B"):
        y = S.unpack(S.sm_packed(packed, n, 5, variant=variant), n)
        assert np.max(np.abs(y - S.softmax(x))) < 1e-12
    with pytest.raises(ValueError):
        S.pack(x[:L // 2], m, slots)             # too few vectors for m ciphertexts


def test_padded_packing_round_trip():
    # n = 200 packed as 256: coordinates 200..255 hold the pad value
    n, slots, m = 200, 1 << 12, 4
    L = m * slots // 256
    x = np.random.default_rng(9).uniform(-64, 0, (L, n))
    p = S.pack(x, m, slots, pad_value=-64.0)
    per = 256 // m
    assert np.all(p[3, (200 - 3 * per) * L:] == -64.0) and np.all(p[:3] > -64.0 - 1e-9)
    assert np.array_equal(S.unpack(p, n), x)


@pytest.mark.parametrize("t", [2, 3, 4])
def test_power_loop_identity(t):
    # SM(x) = normalize(SM(x / t)^t) applied k times: exact functions give SM(x)
    rng = np.random.default_rng(t)
    x = rng.uniform(-32, 0, (500, 24))
    for k in (1, 2, 3):
        assert np.max(np.abs(S.power_loop(x, k, t) - S.softmax(x))) < 1e-12
    # one step from SM(x / t) is the appendix's identity itself
    y = S.softmax(x / t) ** t
    assert np.max(np.abs(y / y.sum(axis=-1, keepdims=True) - S.softmax(x))) < 1e-12


@pytest.mark.parametrize("t", [2, 3, 4])
def test_power_sum_range(t):
    # after a t-th power normalisation sum y = 1, so by the power-mean
    # inequality sum y^t lies in [n^-(t-1), 1], with both ends reached
    n = 16
    rng = np.random.default_rng(10 + t)
    y = S.softmax(rng.uniform(-20, 0, (2000, n)))
    s = (y ** t).sum(axis=-1)
    assert np.all(s >= n ** -(t - 1.0) * (1 - 1e-12)) and np.all(s <= 1.0 + 1e-12)
    assert abs((np.full(n, 1.0 / n) ** t).sum() - n ** -(t - 1.0)) < 1e-15


def test_theorem_bound_under_fixed_point_noise():
    n, M, p = 16, 8.0, 40
    k = S.theorem_k(n, M)
    bound, premise = S.theorem_bound(n, k, p)
    assert premise
    rng = np.random.default_rng(5)
    x = rng.uniform(-M, 0, (2000, n))
    eps = 2.0 ** -p
    exp_noisy = lambda t: np.exp(t) + rng.uniform(-eps, eps, t.shape)
    inv_noisy = [lambda s: s ** -0.5 + rng.uniform(-eps, eps, s.shape)] * k
    y = S.main_loop(x, k, exp_noisy, inv_noisy, rng=rng, eps=eps)
    err = np.max(np.abs(y - S.softmax(x)))
    assert err <= bound
    # heuristic loss of about log M + 1.5 log n bits (Section 3.2)
    assert -math.log2(err) >= p - (math.log2(M) + 1.5 * math.log2(n)) - 2


def test_precision_metrics():
    ref = np.zeros((4, 2))
    y = np.array([[2 ** -10, 0], [0, 2 ** -12], [2 ** -20, 0], [2 ** -16, 0]])
    r = S.precision_bits(ref, y)
    assert r["worst"] == 10
    assert abs(r["mean"] + math.log2(np.mean([2 ** -10, 2 ** -12, 2 ** -20, 2 ** -16]))) < 1e-12
    assert abs(r["std"] - np.std([-10, -12, -20, -16])) < 1e-12


def test_paper_depth_tables_are_self_consistent():
    t = json.load(open(os.path.join(GOLD, "paper_tables.json")))
    for row in t["tab_depth_aux_thread"]["rows"]:
        first, mid, last = row["invsqrt_depths"]
        a, b = row["total"].split("k")
        a = int(a)
        b = int(b) if b else 0
        for k in range(2, 9):
            assert 2 * k + first + mid * (k - 2) + last == a * k + b
    assert t["tab_SMmany"]["SM_B"][-1] == 414


def test_remez_equioscillates():
    a, b, d = 0.81 / 256, 1.21, 31
    coef, err = P.remez(lambda x: x ** -0.5, lambda x: x ** 0.5, a, b, d)
    g = np.linspace(a, b, 200001)
    E = P.cheb_eval(coef, g, a, b) * np.sqrt(g) - 1
    assert abs(np.max(np.abs(E)) - err) < 1e-3 * err
    # d + 2 alternating extrema of (nearly) equal size
    s = np.sign(E)
    runs = 1 + np.count_nonzero(s[1:] != s[:-1])
    assert runs >= d + 2
    # minimax beats interpolation
    ci = P.cheb_interp(lambda x: x ** -0.5, a, b, d)
    Ei = P.cheb_eval(ci, g, a, b) * np.sqrt(g) - 1
    assert np.max(np.abs(Ei)) > err


def test_cheb_interp_reproduces_polynomials():
    c = np.array([0.5, -1.0, 0.25, 2.0])
    f = lambda x: P.cheb_eval(c, x, -3.0, 1.0)
    assert np.allclose(P.cheb_interp(f, -3.0, 1.0, 3), c, atol=1e-13)
    # exponential: error below 2^-40 with degree 15 on [-128, 0] for k = 5
    e = P.exp_table(128.0, 5, 15)
    g = np.linspace(-128, 0, 10001)
    assert np.max(np.abs(P.cheb_eval(e, g, -128.0, 0.0) - np.exp(g / 32))) < 2 ** -40


@pytest.mark.parametrize("case", [(0, 1, 8, 4.0, 3, (31, 31, 31), 14.0, 0, 0),
                                  (1, 2, 12, 8.0, 2, (15, 15, 31), 16.0, 0, 0),
                                  (0, 2, 16, 8.0, 2, (7, 7, 7), 8.0, 1, 1)],
                         ids=["cube-n8", "padded-n12", "newton-averaging"])
def test_encrypted_schedule_variants_on_toy_ring(case):
    # normalize-and-cube, a padded dimension, and Newton's inverse square root
    # with the averaging mask through the oracle's encrypted schedule: after
    # the exponential the padding coordinates hold 0 and the
    # real ones exp(x / t^k) / n^(1/t) (closed form); the output is the FP64
    # Softmax of the n real coordinates to the bits these degrees reach
    import synthetic
    from oracle import ckks, schedule
    variant, m, n, M, t, dinv, bits_min, nw, mm = case
    opt = dict(power=t, newton_steps=nw, mask_mode=mm)
    p = synthetic.preset("toy12")
    o = ckks.Context(**p)
    o.keygen(98)
    n2 = S.padded(n)
    L = m * o.slots // n2
    x = synthetic.logits_uniform(L, n, M, seed=321)
    packed = S.pack(x, m, o.slots)
    xs = [o.encode_encrypt(packed[j], o.delta * 2.0 / M, p["user_top"], 7 + j) for j in range(m)]
    k = schedule.power_k(n, M, t)
    y0 = schedule.softmax(o, xs, n, M, variant=variant, exp_degree=7, inv_degrees=dinv, debug_stop=0, **opt)
    raw = np.stack([o.decrypt_decode(c).real for c in y0])
    got0 = S.unpack(raw, n2)
    want0 = np.zeros((L, n2))
    want0[:, :n] = np.exp(x / float(t) ** k) * float(n) ** (-1.0 / t)
    assert np.max(np.abs(got0 - want0)) < 2.0 ** -14
    ys = schedule.softmax(o, xs, n, M, variant=variant, exp_degree=7, inv_degrees=dinv, **opt)
    y = S.unpack(np.stack([o.decrypt_decode(c).real for c in ys]), n)
    bits = S.precision_bits(S.softmax(x), y)
    assert bits["worst"] >= bits_min, bits
    assert np.max(np.abs(y.sum(axis=1) - 1.0)) < 2.0 ** -(bits_min - 2)


@pytest.mark.parametrize("variant", [0, 1])
def test_encrypted_schedule_on_toy_ring(variant):
    # The oracle's encrypted schedule (Algorithm SM / version B with the
    # auxiliary thread, oracle/schedule.py) on the toy ring: after the first
    # polynomial the slots hold exp(x / 2^k) / sqrt(n) (closed form), and the
    # decrypted output is the FP64 Softmax to >= 16 bits with rows summing to 1.
    import synthetic
    from oracle import ckks, schedule
    p = synthetic.preset("toy12")
    o = ckks.Context(**p)
    o.keygen(99)
    n, M, m = 16, 8.0, 2
    L = m * o.slots // n
    x = synthetic.logits_uniform(L, n, M, seed=123 + variant)
    packed = S.pack(x, m, o.slots)
    xs = [o.encode_encrypt(packed[j], o.delta * 2.0 / M, p["user_top"], 5 + j) for j in range(m)]
    k = schedule.theorem_k(n, M)
    y0 = schedule.softmax(o, xs, n, M, variant=variant, exp_degree=7, inv_degrees=(15, 15, 31), debug_stop=0)
    got0 = S.unpack(np.stack([o.decrypt_decode(c).real for c in y0]), n)
    assert np.max(np.abs(got0 - np.exp(x / 2.0 ** k) / np.sqrt(n))) < 2.0 ** -20
    ys = schedule.softmax(o, xs, n, M, variant=variant, exp_degree=7, inv_degrees=(15, 15, 31))
    y = S.unpack(np.stack([o.decrypt_decode(c).real for c in ys]), n)
    bits = S.precision_bits(S.softmax(x), y)
    assert bits["worst"] >= 16.0, bits
    assert np.max(np.abs(y.sum(axis=1) - 1.0)) < 2.0 ** -14


def test_newton_inverse_sqrt_error_map():
    # Appendix A: with y sqrt(x) = 1 + e, one step y (3 - x y^2) / 2 leaves
    # 1 - e^2 (3 + e) / 2; the schedule's bound delta -> delta^2 (3 + delta)/2
    # is that map at its worst sign, and two steps from 1/2 stay below the
    # lemma's (4/7) (7/8)^(2^n)
    from oracle import schedule
    x = np.linspace(0.01, 4.0, 1001)
    for e in (-0.4, -0.1, 0.05, 0.3):
        y = (1 + e) / np.sqrt(x)
        y1 = y * (3 - x * y * y) / 2
        assert np.allclose(y1 * np.sqrt(x) - 1, -e * e * (3 + e) / 2, atol=1e-14)
        assert abs(e * e * (3 + e) / 2) <= schedule.newton_delta(abs(e), 1) + 1e-17
    d = 0.5
    for steps in (1, 2, 3):
        assert schedule.newton_delta(d, steps) <= 4 / 7 * (7 / 8) ** (2 ** steps)


def test_weighted_minimax_closed_forms():
    # e = 1: min over degree-d P of max |s P(s) - 1| on [a, b] is
    # 1 / T_(d+1)((b + a) / (b - a)) (the Chebyshev polynomial extremal
    # property), reached on the grid up to its spacing
    from oracle import polyeval as PE
    a, b = 0.01, 1.0
    g = np.linspace(a, b, 400001)
    for d in (1, 3, 7, 15):
        c = np.array(PE.minimax_invpow(a, b, d, 1.0))
        err = np.max(np.abs(P.cheb_eval(c, g, a, b) * g - 1))
        want = 1.0 / np.cosh((d + 1) * np.arccosh((b + a) / (b - a)))
        assert abs(err / want - 1) < 1e-6, (d, err, want)
    # degree 0, e = 1/2: the constant 2 / (sqrt(a) + sqrt(b)), relative error
    # (sqrt(b) - sqrt(a)) / (sqrt(b) + sqrt(a)) at both ends
    for a, b in ((1 / 256, 1.0), (0.3, 2.5)):
        c = PE.minimax_invpow(a, b, 0, 0.5)
        assert abs(c[0] - 2 / (math.sqrt(a) + math.sqrt(b))) < 1e-15


def test_weighted_minimax_equioscillates_and_beats_interpolation():
    from oracle import polyeval as PE
    for (a, b, d, e) in ((0.98 / 256, 1.0001, 15, 0.5), (0.98 / 256, 2.0, 31, 0.25), (0.3, 1.3, 7, 1 / 3)):
        c = np.array(PE.minimax_invpow(a, b, d, e))
        g = a + (b - a) * (1 - np.cos(np.linspace(0, np.pi, 200001))) / 2
        E = P.cheb_eval(c, g, a, b) * g ** e - 1
        emax = np.max(np.abs(E))
        # d + 2 alternating extrema of equal size (the minimax on the grid of
        # 16 points per degree: its extrema between grid points exceed the
        # levelled error by well under 1%)
        ext = []
        start = 0
        s = E >= 0
        for i in range(1, len(E) + 1):
            if i == len(E) or s[i] != s[start]:
                ext.append(np.max(np.abs(E[start:i])))
                start = i
        assert len(ext) >= d + 2, (d, len(ext))
        assert min(sorted(ext)[-(d + 2):]) > emax * (1 - 1e-2), (d, e)
        ci = P.cheb_interp(lambda x: x ** -e, a, b, d)
        ei = np.max(np.abs(P.cheb_eval(ci, g, a, b) * g ** e - 1))
        assert emax < ei, (d, e, emax, ei)


def test_packed_jobs_schedule_on_toy_ring():
    # Version B with the jobs' auxiliary ciphertexts packed into one (Section
    # 4.2's single auxiliary ciphertext, across two jobs): each job's
    # decrypted output is the FP64 Softmax of its own logits to the bits its
    # degree-31 polynomial reaches at k = 1 (the toy ring has no bootstrap,
    # and the packing takes two levels per iteration), rows summing to 1, and
    # agrees with the job run alone (its own auxiliary ciphertext) far below
    # that; the jobs' logits differ, so a packing that mixed them up would
    # fail both checks
    import synthetic
    from oracle import ckks, schedule
    p = synthetic.preset("toy12")
    o = ckks.Context(**p)
    o.keygen(97)
    n, M, m, J = 16, 4.0, 2, 2
    L = m * o.slots // n
    xs, cts = [], []
    for jb in range(J):
        x = synthetic.logits_uniform(L, n, M, seed=140 + jb)
        xs.append(x)
        packed = S.pack(x, m, o.slots)
        cts += [o.encode_encrypt(packed[i], o.delta * 2.0 / M, p["user_top"], 60 + jb * m + i) for i in range(m)]
    kw = dict(variant=1, exp_degree=7, inv_degrees=(31, 31, 31))
    ys = schedule.softmax(o, cts, n, M, jobs=J, merge=True, **kw)
    assert len(ys) == J * m
    for jb in range(J):
        y = S.unpack(np.stack([o.decrypt_decode(c).real for c in ys[jb * m:(jb + 1) * m]]), n)
        bits = S.precision_bits(S.softmax(xs[jb]), y)
        assert bits["worst"] >= 14.0, (jb, bits)
        assert np.max(np.abs(y.sum(axis=1) - 1.0)) < 2.0 ** -12
        alone = schedule.softmax(o, cts[jb * m:(jb + 1) * m], n, M, **kw)
        ya = S.unpack(np.stack([o.decrypt_decode(c).real for c in alone]), n)
        assert np.max(np.abs(y - ya)) < 2.0 ** -22, jb
