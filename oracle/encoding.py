"""CKKS slot encoding for the oracle (canonical embedding, special FFT).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Slots: slot j of a real polynomial m holds m(zeta^(5^j mod 2N)), zeta =
exp(i pi / N), j < N0 = N/2 (the paper's N0 slots, Section 2.2).  Writing
w_k = m_k + i m_{k+N0}, the slot vector is z = U w with U[j,k] =
zeta^(5^j k); U^-1 = conj(U)^T / N0.  Decoding evaluates U w with the radix-2
"special FFT" (bit reversal, then log N0 butterfly stages); encoding runs the
same butterflies backwards.

Encoding is specified to the last bit so two implementations agree:
  * twiddles zeta^e are the correctly rounded doubles of (cos, sin)(pi e/N),
    computed here with mpmath's cospi at 160 bits (so cos(pi/2) is exactly 0);
  * butterfly (a, b) -> (a + b, (a - b) * conj(W)), with
    (x * conj(W)).re = x.re*c + x.im*s and .im = x.im*c - x.re*s, each product
    and each sum a separately rounded IEEE double operation (no FMA);
  * after bit reversal the vector is multiplied by 2^-log2(N0) (exact);
  * coefficients are rint(Delta * w) (one rounded product, ties to even).
"""
import functools

import mpmath
import numpy as np


@functools.lru_cache(maxsize=8)
def twiddles(N):
    """(cos, sin)(pi e / N) for e in [0, 2N), correctly rounded doubles."""
    with mpmath.workprec(160):
        quarter = N // 2
        c = np.empty(quarter + 1)
        for e in range(quarter + 1):
            c[e] = float(mpmath.cospi(mpmath.mpf(e) / N))
    cos = np.empty(2 * N)
    sin = np.empty(2 * N)
    for e in range(2 * N):
        if e <= quarter:                       # [0, pi/2]
            cr, sr = c[e], c[quarter - e]
        elif e <= N:                           # (pi/2, pi]: pi/2 + phi
            f = e - quarter
            cr, sr = -c[quarter - f], c[f]
        elif e <= N + quarter:                 # (pi, 3pi/2]: pi + phi
            f = e - N
            cr, sr = -c[f], -c[quarter - f]
        else:                                  # (3pi/2, 2pi): 3pi/2 + phi
            f = e - N - quarter
            cr, sr = c[quarter - f], -c[f]
        cos[e], sin[e] = cr, sr
    return cos, sin


def _brv_perm(n):
    bits = n.bit_length() - 1
    idx = np.arange(n)
    r = np.zeros(n, dtype=np.int64)
    for b in range(bits):
        r |= ((idx >> b) & 1) << (bits - 1 - b)
    return r


def _stage_index(N, length):
    """Twiddle exponents e_j = (5^j mod 4len) * (2N / 4len), j < len/2."""
    h = length // 2
    lq = 4 * length
    e = np.empty(h, dtype=np.int64)
    p = 1
    for j in range(h):
        e[j] = p * (2 * N // lq)
        p = p * 5 % lq
    return e


def special_fft_inverse(N, re, im):
    """w = U^-1 z for z = re + i im of length N/2 (encode direction)."""
    n = N // 2
    cos, sin = twiddles(N)
    vr = np.array(re, dtype=np.float64).copy()
    vi = np.array(im, dtype=np.float64).copy()
    length = n
    while length >= 2:
        h = length // 2
        e = _stage_index(N, length)
        c = cos[e]
        s = sin[e]
        ar = vr.reshape(-1, length)[:, :h]
        ai = vi.reshape(-1, length)[:, :h]
        br = vr.reshape(-1, length)[:, h:]
        bi = vi.reshape(-1, length)[:, h:]
        ur = ar + br
        ui = ai + bi
        dr = ar - br
        di = ai - bi
        tr = dr * c + di * s
        ti = di * c - dr * s
        vr = np.concatenate([ur, tr], axis=1).reshape(-1)
        vi = np.concatenate([ui, ti], axis=1).reshape(-1)
        length //= 2
    perm = _brv_perm(n)
    vr = vr[perm]
    vi = vi[perm]
    scale = 1.0 / n
    return vr * scale, vi * scale


def special_fft(N, wr, wi):
    """z = U w (decode direction)."""
    n = N // 2
    cos, sin = twiddles(N)
    perm = _brv_perm(n)
    vr = np.array(wr, dtype=np.float64)[perm].copy()
    vi = np.array(wi, dtype=np.float64)[perm].copy()
    length = 2
    while length <= n:
        h = length // 2
        e = _stage_index(N, length)
        c = cos[e]
        s = sin[e]
        ar = vr.reshape(-1, length)[:, :h]
        ai = vi.reshape(-1, length)[:, :h]
        br = vr.reshape(-1, length)[:, h:]
        bi = vi.reshape(-1, length)[:, h:]
        tr = br * c - bi * s
        ti = br * s + bi * c
        vr = np.concatenate([ar + tr, ar - tr], axis=1).reshape(-1)
        vi = np.concatenate([ai + ti, ai - ti], axis=1).reshape(-1)
        length *= 2
    return vr, vi


def encode_coeffs(N, z, delta):
    """Integer coefficients (Python ints) of the encoding of z at scale delta."""
    z = np.asarray(z, dtype=np.complex128)
    n = N // 2
    if z.shape[0] != n:
        raise ValueError("expected %d slots" % n)
    wr, wi = special_fft_inverse(N, z.real.copy(), z.imag.copy())
    d = np.float64(delta)
    cr = np.rint(d * wr)
    ci = np.rint(d * wi)
    return [int(v) for v in cr] + [int(v) for v in ci]


def decode_coeffs(N, coeffs, scale):
    """Slots of the real polynomial with integer (or float) coefficients."""
    n = N // 2
    a = np.array([float(c) for c in coeffs], dtype=np.float64) / scale
    zr, zi = special_fft(N, a[:n], a[n:])
    return zr + 1j * zi


def decode_direct(N, coeffs, scale):
    """O(N^2) evaluation of m(zeta^(5^j)) -- the definition, for pinning."""
    n = N // 2
    M = 2 * N
    a = np.array([float(c) for c in coeffs], dtype=np.float64) / scale
    out = np.empty(n, dtype=np.complex128)
    k = np.arange(N)
    p = 1
    for j in range(n):
        e = (p * k) % M
        out[j] = np.sum(a * np.exp(1j * np.pi * e / N))
        p = p * 5 % M
    return out
