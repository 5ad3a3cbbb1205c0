"""Pins of the CKKS oracle: encoding against the O(N^2) definition of the
canonical embedding, decryption of every homomorphic operation against the
plain operation on the slots, rescale against big-integer rounding, and
ModRaise against its definition (t = m mod q0)."""
import numpy as np
import pytest

from oracle import ckks
from oracle.encoding import (decode_coeffs, decode_direct, encode_coeffs, special_fft,
                             special_fft_inverse, twiddles)
import synthetic


@pytest.fixture(scope="module")
def ctx():
    c = ckks.Context(**synthetic.preset("toy12"))
    N = c.N
    c.keygen(2024, galois=[c.galois_rot(1, N), c.galois_rot(-3, N), c.galois_rot(128, N), 2 * N - 1])
    return c


def test_twiddles_correctly_rounded():
    import mpmath
    cos, sin = twiddles(64)
    with mpmath.workprec(200):
        for e in range(128):
            assert cos[e] == float(mpmath.cos(mpmath.pi * e / 64)) or (e % 32 == 0 and abs(cos[e]) in (0.0, 1.0))
            assert sin[e] == float(mpmath.sin(mpmath.pi * e / 64)) or (e % 32 == 0 and abs(sin[e]) in (0.0, 1.0))


@pytest.mark.parametrize("N", [8, 64, 256])
def test_special_fft_is_canonical_embedding(N):
    rng = np.random.default_rng(N)
    coeffs = rng.integers(-1000, 1000, N)
    z = decode_coeffs(N, coeffs, 1.0)
    zd = decode_direct(N, coeffs, 1.0)
    assert np.max(np.abs(z - zd)) < 1e-9
    wr, wi = special_fft_inverse(N, z.real, z.imag)
    assert np.max(np.abs(wr - coeffs[:N // 2])) < 1e-9
    assert np.max(np.abs(wi - coeffs[N // 2:])) < 1e-9


def test_encode_decode_roundtrip():
    N = 256
    z = np.random.default_rng(1).uniform(-1, 1, N // 2) + 1j * np.random.default_rng(2).uniform(-1, 1, N // 2)
    c = encode_coeffs(N, z, 2.0 ** 30)
    assert all(isinstance(v, int) for v in c)
    assert np.max(np.abs(decode_coeffs(N, c, 2.0 ** 30) - z)) < 2 ** -20


def _z(ctx, seed, cplx=True):
    r = np.random.default_rng(seed)
    z = r.uniform(-1, 1, ctx.slots)
    if cplx:
        z = z + 1j * r.uniform(-1, 1, ctx.slots)
    return z


def test_encrypt_decrypt(ctx):
    z = _z(ctx, 1)
    ct = ctx.encode_encrypt(z, ctx.delta, ctx.L, 5)
    assert np.max(np.abs(ctx.decrypt_decode(ct) - z)) < 2 ** -20
    ct2 = ctx.encode_encrypt(z, ctx.delta, 5, 5)
    assert ct2.level == 5 and np.max(np.abs(ctx.decrypt_decode(ct2) - z)) < 2 ** -20


def test_add_mult_levels(ctx):
    a, b = _z(ctx, 2), _z(ctx, 3)
    ca = ctx.encode_encrypt(a, ctx.delta, ctx.L, 6)
    cb = ctx.encode_encrypt(b, ctx.delta, ctx.L, 7)
    s = ctx.add_ct(ca, cb)
    assert np.max(np.abs(ctx.decrypt_decode(s) - (a + b))) < 2 ** -19
    m = ctx.mult(ca, cb)
    assert m.level == ctx.L - 1              # min(l1, l2) - 1 (Section 2.2, "Levels")
    assert np.max(np.abs(ctx.decrypt_decode(m) - a * b)) < 2 ** -18
    m2 = ctx.mult(m, ctx.mod_drop(ca, m.level))
    assert np.max(np.abs(ctx.decrypt_decode(m2) - a * b * a)) < 2 ** -17


def test_rotation_and_conjugation(ctx):
    z = _z(ctx, 4)
    ct = ctx.encode_encrypt(z, ctx.delta, 10, 8)
    for r in (1, -3, 128):
        out = ctx.decrypt_decode(ctx.rotate(ct, r))
        assert np.max(np.abs(out - np.roll(z, -r))) < 2 ** -18
    assert np.max(np.abs(ctx.decrypt_decode(ctx.conjugate(ct)) - np.conj(z))) < 2 ** -18


def test_plain_and_constant_ops(ctx):
    z, w = _z(ctx, 5), _z(ctx, 6, cplx=False)
    ct = ctx.encode_encrypt(z, ctx.delta, 10, 9)
    pt, _ = ctx.encode(w, float(ctx.q[10]), 10)
    out = ctx.rescale(ctx.mul_plain(ct, pt, float(ctx.q[10])))
    assert np.max(np.abs(ctx.decrypt_decode(out) - z * w)) < 2 ** -18
    out = ctx.mul_int(ct, -3)
    assert np.max(np.abs(ctx.decrypt_decode(out) + 3 * z)) < 2 ** -18
    out = ctx.add_int(ct, int(round(0.25 * ct.scale)))
    assert np.max(np.abs(ctx.decrypt_decode(out) - (z + 0.25))) < 2 ** -19
    # multiplication by X^(N/2) multiplies every slot by i
    out = ctx.mul_monomial(ct, ctx.N // 2)
    assert np.max(np.abs(ctx.decrypt_decode(out) - 1j * z)) < 2 ** -19


def test_rescale_is_rounded_division(ctx):
    z = _z(ctx, 7)
    ct = ctx.encode_encrypt(z, ctx.delta, 3, 10)
    out = ctx.rescale(ct)
    lv = ct.level
    for comp_in, comp_out in zip(ct.c, out.c):
        cin = ctx.crt([ctx.intt(comp_in[i], i) for i in range(lv + 1)], list(range(lv + 1)))
        cout = ctx.crt([ctx.intt(comp_out[i], i) for i in range(lv)], list(range(lv)))
        Q = 1
        for i in range(lv):
            Q *= ctx.q[i]
        ql = ctx.q[lv]
        for k in range(0, ctx.N, 97):
            x = cin[k] % (Q * ql)
            r = x % ql
            if r > (ql - 1) // 2:
                r -= ql
            want = ((x - r) // ql) % Q
            assert cout[k] % Q == want


def test_mod_raise_definition(ctx):
    z = _z(ctx, 8, cplx=False) * 0.01
    ct = ctx.mod_drop(ctx.encode_encrypt(z, ctx.delta, 5, 11), 0)
    m0 = ctx.decrypt_coeffs(ct)
    raised = ctx.mod_raise(ct, 4)
    t = ctx.decrypt_coeffs(raised)
    q0 = ctx.q[0]
    I = [(a - b) // q0 for a, b in zip(t, m0)]
    assert all((a - b) % q0 == 0 for a, b in zip(t, m0))
    # |I| <= (h + 1) / 2 with h the secret weight (uniform ternary: <= N)
    assert max(abs(v) for v in I) <= (np.count_nonzero(ctx.s_coeff) + 1) // 2 + 1
    assert max(abs(v) for v in I) > 0


def test_key_switch_noise_is_small(ctx):
    z = _z(ctx, 9)
    ct = ctx.encode_encrypt(z, ctx.delta, ctx.L, 12)
    m = ctx.decrypt_coeffs(ct)
    g = ctx.galois_rot(1, ctx.N)
    N = ctx.N
    mg = [0] * N
    for j, v in enumerate(m):
        e = j * g % (2 * N)
        if e < N:
            mg[e] += v
        else:
            mg[e - N] -= v
    mr = ctx.decrypt_coeffs(ctx.rotate(ct, 1))
    err = max(abs(a - b) for a, b in zip(mr, mg))
    # ModDown rounding: |u0 + u1 s| <= (alpha + 1) (1 + ||s||_1) / 2
    assert err <= (len(ctx.p) + 1) * (1 + np.count_nonzero(ctx.s_coeff))


def test_hoisted_rotation_is_a_rotation(ctx):
    # one ModUp for several offsets: each result decrypts to the automorphism
    # of the plaintext coefficients (X -> X^g) plus ModDown rounding of the
    # same bound as an ordinary rotation, and its slots are the rotated slots
    z = _z(ctx, 13)
    ct = ctx.encode_encrypt(z, ctx.delta, ctx.L, 14)
    m = ctx.decrypt_coeffs(ct)
    N = ctx.N
    rots = [1, -3, 128]
    for r, h in zip(rots, ctx.rotate_hoisted(ct, rots)):
        g = ctx.galois_rot(r, N)
        mg = [0] * N
        for j, v in enumerate(m):
            e = j * g % (2 * N)
            if e < N:
                mg[e] += v
            else:
                mg[e - N] -= v
        err = max(abs(a - b) for a, b in zip(ctx.decrypt_coeffs(h), mg))
        assert err <= (len(ctx.p) + 1) * (1 + np.count_nonzero(ctx.s_coeff)), (r, err)
        assert np.max(np.abs(ctx.decrypt_decode(h) - np.roll(z, -r))) < 2 ** -18


def test_mod_down_is_rounded_division_by_P(ctx):
    # ModDown of c over Q_l u P: (c - Conv_P->Q([c]_P)) P^-1 = round(c / P) - u
    # with |u| < (alpha + 1) / 2 (the centred conversion's multiple of P),
    # checked by big-integer CRT on random polynomials over Q_l P
    rng = np.random.default_rng(77)
    level = 5
    idx = list(range(level + 1)) + list(range(len(ctx.q), len(ctx.primes)))
    Q = 1
    for i in range(level + 1):
        Q *= ctx.q[i]
    QP = Q * ctx.P
    C = [int.from_bytes(rng.bytes(64), "little") % QP for _ in range(ctx.N)]
    limbs = [ctx.ntt(np.array([x % ctx.primes[t] for x in C], dtype=np.uint64), t) for t in idx]
    out = ctx.mod_down(limbs, level)
    got = ctx.crt([ctx.intt(out[i], i) for i in range(level + 1)], list(range(level + 1)))
    alpha = len(ctx.p)
    worst = 0
    ds = []
    for k in range(ctx.N):
        cp = C[k] % ctx.P
        if cp > ctx.P // 2:
            cp -= ctx.P
        r = (C[k] - cp) // ctx.P             # nearest integer to C / P
        d = (got[k] - r) % Q
        if d > Q // 2:
            d -= Q
        worst = max(worst, abs(d))
        ds.append(d)
    assert worst < (alpha + 1) / 2
    # unbiased: a plain (non-centred) conversion would shift every
    # coefficient by about -(alpha - 1) / 2 on average
    assert abs(np.mean(ds)) < 5 * np.std(ds) / np.sqrt(len(ds)) + 0.02
