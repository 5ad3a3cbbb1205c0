"""Pins of the oracle's bootstrapping (oracle/bootstrap.py) against closed
forms at every stage, on the small bootstrapping ring (N = 2^10):

* after ModRaise the coefficients are t = m' + q0 I with |I| <= K (m' the
  input's coefficients times the integer size factor);
* after CoeffToSlot slot j holds (t_brv(j) + i t_brv(j)+n) / (2 q0 (K+1))
  (the inverse canonical embedding without its bit reversal);
* the real part u_re = t_brv(j) / (q0 (K+1));
* after the polynomial z = exp(2 pi i t / (q0 2^r)), after the r squarings
  exp(2 pi i t / q0);
* the SlotToCoeff input 2 (8 sin x - sin 2x) + 2i (8 sin y - sin 2y) with
  x, y = 2 pi t / q0 of the two halves;
* the output decrypts to the input within 2^-22 (the paper's bootstrapping
  precision, Section 5.1), at several input levels and with the slot mask.
"""
import numpy as np
import pytest

import synthetic

P = synthetic.preset("boot10")


@pytest.fixture(scope="module")
def boot():
    from oracle import ckks
    from oracle.bootstrap import Bootstrapper
    o = ckks.Context(**P)
    o.keygen(808)
    return o, Bootstrapper(o, P["boot"], P["user_top"], P["log_scale"])


def _brv(n):
    b = n.bit_length() - 1
    return np.array([int(format(i, "0%db" % b)[::-1], 2) for i in range(n)])


def _z(o, seed, amp=0.9):
    r = np.random.default_rng(seed)
    return amp * (r.uniform(-1, 1, o.slots) + 1j * r.uniform(-1, 1, o.slots)) / np.sqrt(2)


def test_stages_follow_their_closed_forms(boot):
    o, bs = boot
    K, r = P["boot"]["K"], P["boot"]["double_angle"]
    n = o.slots
    q0 = o.q[0]
    z = _z(o, 1)
    ct = o.encode_encrypt(z, o.delta, 2, 3)
    tr = {}
    out = bs.bootstrap(ct, 1.0, trace=tr)
    # ModRaise: t = m' + q0 I, m' = kf m with the integer size factor kf
    m = o.decrypt_coeffs(o.mod_drop(ct, 0))
    t = o.decrypt_coeffs(tr[1])
    kf = int(min(np.floor(q0 / 512.0 / ct.scale), 16.0))     # bound 1: the size factor rule
    kf = kf if kf >= 2 else 1
    I = [(a - kf * b) // q0 for a, b in zip(t, m)]
    assert all((a - kf * b) % q0 == 0 for a, b in zip(t, m))
    assert max(abs(v) for v in I) <= K and max(abs(v) for v in I) > 0
    tt = np.array([float(v) for v in t])
    brv = _brv(n)
    lo, hi = tt[brv], tt[brv + n]
    # CoeffToSlot
    want2 = (lo + 1j * hi) / (2.0 * q0 * (K + 1))
    assert np.max(np.abs(o.decrypt_decode(tr[2]) - want2)) < 2.0 ** -30
    assert np.max(np.abs(o.decrypt_decode(tr[3]) - lo / (q0 * (K + 1)))) < 2.0 ** -30
    # EvalMod: the polynomial, then the squarings
    want4 = np.exp(2j * np.pi * lo / (q0 * 2.0 ** r))
    assert np.max(np.abs(o.decrypt_decode(tr[4]) - want4)) < 2.0 ** -30
    assert np.max(np.abs(o.decrypt_decode(tr[5]) - np.exp(2j * np.pi * lo / q0))) < 2.0 ** -26
    assert np.max(np.abs(o.decrypt_decode(tr[6]) - np.exp(2j * np.pi * hi / q0))) < 2.0 ** -26
    # the harmonic correction and the recombination
    x, y = 2 * np.pi * lo / q0, 2 * np.pi * hi / q0
    want7 = 2 * (8 * np.sin(x) - np.sin(2 * x)) + 2j * (8 * np.sin(y) - np.sin(2 * y))
    assert np.max(np.abs(o.decrypt_decode(tr[7]) - want7)) < 2.0 ** -24
    # the refreshed message
    assert out.level == P["user_top"]
    assert np.max(np.abs(o.decrypt_decode(out) - z)) < 2.0 ** -22


@pytest.mark.parametrize("level,scale_bits,amp", [(0, 40, 0.9), (3, 40, 0.01), (4, 50, 0.5)])
def test_refresh_any_level(boot, level, scale_bits, amp):
    # the size rule takes both branches: integer factor (small values) and
    # the division by 2^e (a large scale at level >= 1)
    o, bs = boot
    z = _z(o, 10 + level, amp)
    ct = o.encode_encrypt(z, 2.0 ** scale_bits, level, 4)
    out = bs.bootstrap(ct, 1.0)
    assert out.level == P["user_top"]
    assert np.max(np.abs(o.decrypt_decode(out) - z)) < 2.0 ** -22


def test_masked_refresh(boot):
    o, bs = boot
    L = 64
    z = _z(o, 20).real
    ct = o.encode_encrypt(z, o.delta, 1, 5)
    got = o.decrypt_decode(bs.bootstrap(ct, 1.0, mask_L=L))
    want = np.where(np.arange(o.slots) < L, z, 0.0)
    assert np.max(np.abs(got - want)) < 2.0 ** -22
