"""Pins of the ring oracle against definitions that do not come from it:
published Philox known answers, the O(N^2) NTT definition and schoolbook
negacyclic convolution, big-integer CRT, the coefficient-domain automorphism,
primality, and the sampler distributions."""
import os

import numpy as np
import pytest
import sympy

from oracle import _lib
from oracle.params import find_primes, smallest_psi
from oracle import ckks

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _prime(N, bits=40):
    q, _ = find_primes(N.bit_length() - 1, [bits], [])
    return q[0]


def test_philox_known_answers():
    L = _lib.lib()
    rows = [l.split() for l in open(os.path.join(GOLD, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        ctr = np.array([int(v, 16) for v in r[0:4]], dtype=np.uint32)
        key = np.array([int(v, 16) for v in r[4:6]], dtype=np.uint32)
        want = [int(v, 16) for v in r[6:10]]
        out = np.zeros(4, dtype=np.uint32)
        L.or_philox4x32_10(ctr, key, out)
        assert out.tolist() == want


@pytest.mark.parametrize("N", [4, 16, 64, 256])
def test_ntt_matches_definition_and_inverts(N):
    L = _lib.lib()
    for bits in (40, 60):
        q = _prime(N, bits)
        psi = smallest_psi(q, N)
        a = np.random.default_rng(N + bits).integers(0, q, N, dtype=np.uint64)
        d = np.empty(N, dtype=np.uint64)
        L.or_ntt_definition(a, d, N, q, psi)
        pb = np.empty(N, dtype=np.uint64)
        pib = np.empty(N, dtype=np.uint64)
        L.or_psi_tables(N, q, psi, pb, pib)
        f = a.copy()
        L.or_ntt_fwd(f, N, q, pb)
        assert np.array_equal(f, d)
        L.or_ntt_inv(f, N, q, pib)
        assert np.array_equal(f, a)
        # the definition itself: evaluation at psi^(2 brv(i) + 1), by Horner in Python
        lg = N.bit_length() - 1
        for i in (0, 1, N - 1):
            e = 2 * int(format(i, "0%db" % lg)[::-1], 2) + 1 if lg else 1
            x = pow(psi, e, q)
            acc = 0
            for c in reversed(a.tolist()):
                acc = (acc * x + c) % q
            assert acc == int(d[i])


@pytest.mark.parametrize("N", [8, 64, 512])
def test_ntt_convolution_theorem(N):
    L = _lib.lib()
    q = _prime(N)
    psi = smallest_psi(q, N)
    pb = np.empty(N, dtype=np.uint64)
    pib = np.empty(N, dtype=np.uint64)
    L.or_psi_tables(N, q, psi, pb, pib)
    rng = np.random.default_rng(N)
    a = rng.integers(0, q, N, dtype=np.uint64)
    b = rng.integers(0, q, N, dtype=np.uint64)
    school = np.empty(N, dtype=np.uint64)
    L.or_negacyclic_mul(a, b, school, N, q)
    # schoolbook again, in Python big integers, for the first coefficients
    for k in (0, 1, N - 1):
        s = 0
        for i in range(N):
            j = k - i
            if j >= 0:
                s += int(a[i]) * int(b[j])
            else:
                s -= int(a[i]) * int(b[j + N])
        assert s % q == int(school[k])
    fa, fb = a.copy(), b.copy()
    L.or_ntt_fwd(fa, N, q, pb)
    L.or_ntt_fwd(fb, N, q, pb)
    prod = np.empty(N, dtype=np.uint64)
    L.or_vec_mul(fa, fb, prod, N, q)
    L.or_ntt_inv(prod, N, q, pib)
    assert np.array_equal(prod, school)


def test_primes_and_psi():
    for logN, bits in [(12, [40] * 24 + [60] * 2), (16, [52, 40, 40, 50, 58])]:
        N = 1 << logN
        q, p = find_primes(logN, bits[:-2], bits[-2:])
        allp = q + p
        assert len(set(allp)) == len(allp)
        for t, b in zip(allp, bits):
            assert sympy.isprime(t)
            assert t % (2 * N) == 1
            assert abs(t.bit_length() - b) <= 1 and abs(t - 2 ** b) < 2 ** (b - 8)
        for t in allp[:3]:
            psi = smallest_psi(t, N)
            assert pow(psi, N, t) == t - 1
            # smallest: no smaller x of order 2N among a sample of small x
            for x in range(2, min(psi, 2000)):
                assert pow(x, N, t) != t - 1


def test_base_conversion_against_crt():
    N = 16
    q, p = find_primes(4, [40, 40, 40], [60, 60])
    L = _lib.lib()
    rng = np.random.default_rng(3)
    src, dst = q, p
    D = 1
    for d in src:
        D *= d
    X = [int(v) for v in rng.integers(0, 2 ** 62, N)]
    X = [(x * 12345678901234567) % D for x in X]
    inp = np.array([[x % d for x in X] for d in src], dtype=np.uint64).reshape(-1)
    out = np.empty(len(dst) * N, dtype=np.uint64)
    L.or_base_convert(inp, np.array(src, dtype=np.uint64), len(src), out,
                      np.array(dst, dtype=np.uint64), len(dst), N)
    out = out.reshape(len(dst), N)
    for c in range(N):
        # y_t = (X + u D) mod t with u in [0, |src|)
        ok = False
        for u in range(len(src)):
            if all(int(out[t][c]) == (X[c] + u * D) % dst[t] for t in range(len(dst))):
                ok = True
        assert ok


def test_automorphism_perm_matches_coefficient_map():
    N = 64
    L = _lib.lib()
    q = _prime(N)
    psi = smallest_psi(q, N)
    pb = np.empty(N, dtype=np.uint64)
    pib = np.empty(N, dtype=np.uint64)
    L.or_psi_tables(N, q, psi, pb, pib)
    a = np.random.default_rng(9).integers(0, q, N, dtype=np.uint64)
    for g in (5, 25, 2 * N - 1, pow(5, 7, 2 * N)):
        # coefficient domain: a(X^g)
        ag = [0] * N
        for j in range(N):
            e = j * g % (2 * N)
            if e < N:
                ag[e] = (ag[e] + int(a[j])) % q
            else:
                ag[e - N] = (ag[e - N] - int(a[j])) % q
        fa = a.copy()
        L.or_ntt_fwd(fa, N, q, pb)
        fag = np.array(ag, dtype=np.uint64)
        L.or_ntt_fwd(fag, N, q, pb)
        perm = np.empty(N, dtype=np.uint64)
        L.or_automorph_perm(N, g, perm)
        assert np.array_equal(fa[perm.astype(np.int64)], fag)


def test_samplers():
    L = _lib.lib()
    N = 1 << 14
    t = np.empty(N, dtype=np.int64)
    L.or_sample_ternary(7, 1, N, t)
    assert set(np.unique(t).tolist()) == {-1, 0, 1}
    assert abs(np.mean(t == 0) - 1 / 3) < 0.02
    L.or_sample_sparse_ternary(7, 2, N, 192, t)
    assert np.count_nonzero(t) == 192 and set(np.unique(t).tolist()) <= {-1, 0, 1}
    cdt = ckks.gaussian_cdt(3.2)
    assert np.all(np.diff(cdt.astype(object)) >= 0)
    # Pr(e = 0) = 1 / sum_k exp(-k^2 / (2 sigma^2)) (theta function, ~0.1245)
    z = sum(np.exp(-(k * k) / (2 * 3.2 ** 2)) for k in range(-60, 61))
    assert abs(int(cdt[0]) / 2 ** 64 - 1 / z) < 1e-15
    L.or_sample_cdt(7, 3, N, cdt, len(cdt), t)
    assert abs(t.var() - 3.2 ** 2) < 0.5 and abs(t.mean()) < 0.1
    u = np.empty(N, dtype=np.uint64)
    q = _prime(N, 50)
    L.or_sample_uniform(7, 4, N, q, u)
    assert u.max() < q and abs(u.astype(np.float64).mean() / q - 0.5) < 0.02
    # 128-bit reduction, checked against Python big integers
    w = np.zeros(4, dtype=np.uint32)
    L.or_draw_block(7, 4, 5, w)
    v = sum(int(w[i]) << (32 * i) for i in range(4))
    assert v % q == int(u[5])


def _conv(fn, X, src, dst, N):
    L = _lib.lib()
    inp = np.array([[x % d for x in X] for d in src], dtype=np.uint64).reshape(-1)
    out = np.empty(len(dst) * N, dtype=np.uint64)
    getattr(L, fn)(inp, np.array(src, dtype=np.uint64), len(src), out, np.array(dst, dtype=np.uint64), len(dst), N)
    return out.reshape(len(dst), N)


def _lift_multiple(out, c, X, D, dst, umax):
    """The integer u in [-umax, umax] with out[t][c] = (X + u D) mod t for every
    target t (None when there is none: then no integer congruent to X mod D
    with that bound explains the output)."""
    hits = [u for u in range(-umax, umax + 1) if all(int(out[t][c]) == (X + u * D) % dst[t] for t in range(len(dst)))]
    return hits[0] if len(hits) == 1 else None


@pytest.mark.parametrize("k", [2, 3, 5])
def test_centred_base_conversion_against_crt(k):
    # The centred conversion (used by ModDown) takes each [x_i (D/d_i)^-1]_{d_i}
    # in (-d_i/2, d_i/2]: its output is the residue of an integer X_c + u D
    # (X_c the centred representative of X mod D) with |u| < (k + 1) / 2 and
    # u of mean zero; the plain conversion gives X + u D with 0 <= u < k.
    # Checked by big-integer CRT on every coefficient.
    N = 256
    q, p = find_primes(8, [40] * k, [60] * 3)
    src, dst = q, p
    D = 1
    for d in src:
        D *= d
    rng = np.random.default_rng(30 + k)
    X = [int.from_bytes(rng.bytes(40), "little") % D for _ in range(N)]
    out_c = _conv("or_base_convert_centered", X, src, dst, N)
    out_p = _conv("or_base_convert", X, src, dst, N)
    uc, up = [], []
    for c in range(N):
        xc = X[c] - D if X[c] > D // 2 else X[c]
        u = _lift_multiple(out_c, c, xc, D, dst, k + 1)
        assert u is not None and abs(u) < (k + 1) / 2, (c, u)
        uc.append(u)
        u = _lift_multiple(out_p, c, X[c], D, dst, k + 1)
        assert u is not None and 0 <= u < k, (c, u)
        up.append(u)
    # zero mean (the centred terms are symmetric): |mean| within 5 standard
    # errors; the plain conversion's u has mean about (k - 1) / 2
    sd = np.std(uc) / np.sqrt(N) + 1e-9
    assert abs(np.mean(uc)) < 5 * sd + 0.05
    assert np.mean(up) > (k - 1) / 2 - 0.5


def test_centred_base_conversion_tie_rule():
    # (-d/2, d/2] for odd d: the residue (d - 1) / 2 stays positive and
    # (d + 1) / 2 becomes -(d - 1) / 2.  X is built from chosen lifted terms
    # xh_i = [x_i (D/d_i)^-1]_{d_i}, so the exact integer the conversion must
    # reproduce is sum_i xh_i' D / d_i with xh_i' the centred xh_i.
    N = 4
    src, dst = find_primes(4, [40, 40, 40], [60, 60])
    D = 1
    for d in src:
        D *= d
    choices = [((src[0] - 1) // 2, 5, 0), ((src[0] + 1) // 2, 7, 1), (1, (src[1] - 1) // 2, (src[2] + 1) // 2),
               (src[0] - 1, src[1] - 1, src[2] - 1)]
    X, want = [], []
    for xh in choices:
        x = 0
        s = 0
        for i, d in enumerate(src):
            Di = D // d
            x += xh[i] * Di          # x_i = xh_i (D/d_i) mod d_i
            s += (xh[i] - d if xh[i] > (d - 1) // 2 else xh[i]) * Di
        X.append(x % D)
        want.append(s)
    out = _conv("or_base_convert_centered", X, src, dst, N)
    for c in range(N):
        for t in range(len(dst)):
            assert int(out[t][c]) == want[c] % dst[t], (c, t)
