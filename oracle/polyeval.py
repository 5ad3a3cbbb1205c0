"""Homomorphic polynomial evaluation on oracle ciphertexts: Chebyshev
approximations evaluated by baby-step giant-step with exact scales.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper evaluates its auxiliary functions (the exponential, x^(-1/2),
x^(-2^-j)) as polynomials of degree 2^t - 1 in about log2 of the degree
levels with O(sqrt(degree)) ciphertext products (Section 2.2, "Functions as
polynomials", Paterson-Stockmeyer), with coefficients from a minimax fit
(Section 5.1, "Designing auxiliary functions").  It prints neither the
coefficients nor the evaluation order, so this module states one and the
HIP library implements the same one (scale-exact baby-step giant-step in
the Chebyshev basis, Bossuat et al., EUROCRYPT 2021):

* coefficients: for the exponential, the interpolant at the d+1 Chebyshev
  nodes of the first kind of [a, b], computed in mpmath at 256 bits and
  rounded once to double (``cheb_interp``); for the inverse powers s^-e,
  the paper's weighted minimax approximant (min max |P(s) s^e - 1|), as the
  discrete minimax on a fixed grid by the Remez exchange
  (``minimax_invpow``, steps stated there);
* the argument u = alpha x + beta maps [a, b] to [-1, 1]: alpha = 2/(b-a) and
  beta = -(a+b)/(b-a) as doubles; when alpha is a power of two >= 1 it is an
  integer product (no level), else a constant product at scale 2^log_scale;
  then beta is added;
* with t = ceil(log2(d+1)) the result sits t+1 levels below u, and the
  baby-step size is B = 2^max(1, floor((t+1)/2));
* eval(c, S, l): if deg c < B it is a leaf; else with n the largest power of
  two B 2^i <= deg, c = c_lo + c_hi T_n (T_(n+k) = 2 T_n T_k - T_(n-k)):
  c_hi = (c_n, 2 c_(n+1), ..., 2 c_deg), c_lo = c_0..c_(n-1) minus c_(n+k) at
  n-k; the high part is evaluated at (S q_(l+1) / scale(T_n), l+1), times
  T_n (dropped to level l+1) and rescaled, declared scale S; the low part
  at (S, l) is added;
* a leaf sum_j c_j T_j at (S, l): every T_j (read at level l+1) is multiplied
  by the integer rint(c_j (S q_(l+1)) / scale(T_j)) (terms rounding to 0 are
  dropped), the products are summed, rint(c_0 S q_(l+1)) is added to the
  first component, one rescale, declared scale S.  Imaginary parts of
  complex coefficients are summed apart and multiplied by X^(N/2) (times i on
  every slot);
* T_1 = u; T_2k = 2 T_k^2 - 1; T_2k+1 = 2 T_(k+1) T_k - T_1, the product of
  two operands at different levels taken at the lower one, and T_1 there
  brought to that level and exact scale by a constant product by 1.0;
* a constant term c of a high part that reduced to a constant is a constant
  product of T_n to the scale S (real and imaginary parts apart);
* with a slot mask (a 0/1 slot vector mu): every constant c is replaced by
  the plaintext rint(c s mu) at the scale s it enters with, which multiplies
  the whole polynomial by mu (mu^2 = mu) at no extra level.

Every floating-point step above is one IEEE double operation in the order
written, so the integer constants, and with them the ciphertexts, are the
same as the library's bit for bit.
"""
import math

import mpmath
import numpy as np

from .ckks import Ciphertext
from .encoding import special_fft_inverse


def cheb_interp(f, a, b, d, prec=256):
    """Chebyshev interpolant of f (an mpmath function) on [a, b] at the d+1
    first-kind nodes, coefficients rounded to double."""
    with mpmath.workprec(prec):
        a_, b_ = mpmath.mpf(a), mpmath.mpf(b)
        nodes = [mpmath.cos(mpmath.pi * (k + mpmath.mpf(1) / 2) / (d + 1)) for k in range(d + 1)]
        fx = [f((u * (b_ - a_) + a_ + b_) / 2) for u in nodes]
        out = []
        for j in range(d + 1):
            s = mpmath.fsum(fx[k] * mpmath.cos(mpmath.pi * j * (k + mpmath.mpf(1) / 2) / (d + 1))
                            for k in range(d + 1))
            cj = 2 * s / (d + 1)
            if j == 0:
                cj /= 2
            out.append(float(cj))
    return out


_MINIMAX = {}


def _solve_ld(A, y):
    """Gaussian elimination with partial pivoting (numpy long double)."""
    A = A.copy()
    y = y.copy()
    n = len(y)
    for col in range(n):
        piv = col + int(np.argmax(np.abs(A[col:, col])))
        if piv != col:
            A[[col, piv]] = A[[piv, col]]
            y[[col, piv]] = y[[piv, col]]
        f = A[col + 1:, col] / A[col, col]
        A[col + 1:, col:] -= np.outer(f, A[col, col:])
        y[col + 1:] -= f * y[col]
    x = np.zeros(n, dtype=np.longdouble)
    for r in range(n - 1, -1, -1):
        x[r] = (y[r] - np.dot(A[r, r + 1:], x[r + 1:])) / A[r, r]
    return x


def minimax_invpow(a, b, d, e):
    """Weighted minimax approximant of s^-e on [a, b] (Section 5.1, "Designing
    auxiliary functions": the polynomial P of degree d with the smallest
    max |P(s) s^e - 1|), coefficients in the Chebyshev basis of [a, b].

    Computed as the minimax on the grid u_i = -cos(pi i / (G - 1)),
    i = 0..G-1, G = 16 (d + 1) + 1, by the Remez exchange:
    * reference: the grid indices 16 k, k = 0..d+1 (the extrema of T_(d+1));
    * each round (at most 40, in 80-bit long double): solve
      sum_j c_j T_j(u_k) + (-1)^k h / w_k = 1 / w_k at the reference
      (w = s^e); with r = w P - 1 on the grid, take in every run of equal
      sign (r >= 0 counting as positive) the index of the largest |r| (the
      first on ties); while more than d + 2 remain, drop the end one with the
      smaller |r| (the last on ties); stop when fewer remain or nothing
      changed, else take them as the new reference; stop before the exchange
      when the levelled error |h| is below 2^-40 (far below any ciphertext's
      precision, and near the rounding of r in long double, where the
      exchange would follow noise);
    * the coefficients: the reference system solved again at 50 decimal
      digits (mpmath), each rounded to the nearest multiple of 2^(E - 52)
      with 2^E <= max |c_j| < 2^(E+1) (the largest one's double ulp), so
      that the small high-order coefficients of a near-exact fit are as
      reproducible as the largest.
    Test infrastructure: cached per (a, b, d, e)."""
    key = (float(a), float(b), int(d), float(e))
    if key in _MINIMAX:
        return list(_MINIMAX[key])
    G = 16 * (d + 1) + 1
    pi = np.longdouble("3.14159265358979323846264338327950288")
    al, bl, el = np.longdouble(a), np.longdouble(b), np.longdouble(e)
    u = -np.cos(pi * np.arange(G, dtype=np.longdouble) / np.longdouble(G - 1))
    s = (u * (bl - al) + al + bl) / 2
    w = np.power(s, el)
    T = np.empty((G, d + 1), dtype=np.longdouble)
    T[:, 0] = 1
    if d >= 1:
        T[:, 1] = u
    for j in range(2, d + 1):
        T[:, j] = 2 * u * T[:, j - 1] - T[:, j - 2]
    sgn = np.array([(-1) ** k for k in range(d + 2)], dtype=np.longdouble)
    ref = [16 * k for k in range(d + 2)]
    for _ in range(40):
        A = np.concatenate([T[ref], (sgn / w[ref])[:, None]], axis=1)
        sol = _solve_ld(A, 1 / w[ref])
        if abs(sol[d + 1]) < np.longdouble(2.0) ** -40:
            break
        c = sol[:d + 1]
        r = w * (T @ c) - 1
        pos = r >= 0
        cand = []
        start = 0
        for i in range(1, G + 1):
            if i == G or pos[i] != pos[start]:
                cand.append(start + int(np.argmax(np.abs(r[start:i]))))
                start = i
        while len(cand) > d + 2:
            if abs(r[cand[0]]) < abs(r[cand[-1]]):
                cand.pop(0)
            else:
                cand.pop()
        if len(cand) < d + 2 or cand == ref:
            break
        ref = cand
    with mpmath.workdps(50):
        a_, b_, e_ = mpmath.mpf(a), mpmath.mpf(b), mpmath.mpf(e)
        rows, rhs = [], []
        for k, i in enumerate(ref):
            uk = -mpmath.cos(mpmath.pi * i / (G - 1))
            sk = (uk * (b_ - a_) + a_ + b_) / 2
            wk = mpmath.power(sk, e_)
            t = [mpmath.mpf(1), uk]
            while len(t) < d + 1:
                t.append(2 * uk * t[-1] - t[-2])
            rows.append(t[:d + 1] + [(-1) ** k / wk])
            rhs.append(1 / wk)
        sol = mpmath.lu_solve(mpmath.matrix(rows), mpmath.matrix(rhs))
        cmax = max(abs(sol[j]) for j in range(d + 1))
        E = int(mpmath.floor(mpmath.log(cmax, 2)))
        if mpmath.ldexp(1, E) > cmax:       # log rounding at a power of two
            E -= 1
        elif mpmath.ldexp(1, E + 1) <= cmax:
            E += 1
        unit = mpmath.ldexp(1, E - 52)
        out = [float(mpmath.nint(sol[j] / unit) * unit) for j in range(d + 1)]
    _MINIMAX[key] = out
    return list(out)


def cheb_eval_plain(coef, a, b, x):
    """Clenshaw evaluation in double, operation by operation."""
    u = (2 * x - a - b) / (b - a)
    b1 = 0.0
    b2 = 0.0
    for j in range(len(coef) - 1, 0, -1):
        t = 2 * u * b1 - b2 + coef[j]
        b2 = b1
        b1 = t
    return u * b1 - b2 + coef[0]


def ceil_log2(x):
    l = 0
    while (1 << l) < x:
        l += 1
    return l


def depth(degree):
    """Levels used by the evaluation (without the affine map)."""
    return ceil_log2(degree + 1) + 1


# --------------------------------------------------------------- ring helpers
def drop(ctx, a, level):
    return a if a.level == level else ctx.mod_drop(a, level)


def mult(ctx, a, b):
    """Tensor, relinearise, rescale; operands at different levels are taken
    at the lower one."""
    lv = min(a.level, b.level)
    return ctx.mult(drop(ctx, a, lv), drop(ctx, b, lv))


def mul_const(ctx, a, v, target_scale):
    """a times the constant v with the result at exactly target_scale: the
    integer K = rint(v (target q_l / scale(a))), one rescale."""
    S = target_scale * float(ctx.q[a.level]) / a.scale
    K = int(np.rint(v * S))
    out = ctx.rescale(ctx.mul_int(a, K))
    out.scale = target_scale
    return out


def add_const(ctx, a, v):
    """a plus the constant v: rint(v scale(a)) on the first component."""
    return ctx.add_int(a, int(np.rint(v * a.scale)))


def scale_int(ctx, a, k):
    """a times the integer k (scale unchanged)."""
    return ctx.mul_int(a, k)


class Mask:
    """A 0/1 slot vector mu as plaintexts rint(s w) (w its encoding's real
    coefficients, the inverse special FFT of mu) at any scale s."""

    def __init__(self, ctx, slots01):
        self.ctx = ctx
        N = ctx.N
        wr, wi = special_fft_inverse(N, np.asarray(slots01, dtype=np.float64), np.zeros(N // 2))
        self.w = np.concatenate([wr, wi])

    def plaintext(self, s, level):
        coeffs = [int(v) for v in np.rint(np.float64(s) * self.w)]
        return [self.ctx.ntt(self.ctx.ints_to_limb(coeffs, i), i) for i in range(level + 1)]

    def add(self, a, v):
        """a plus rint(v scale(a) w) on the first component."""
        pt = self.plaintext(v * a.scale, a.level)
        c0 = np.stack([self.ctx.add(a.c[0][i], pt[i], i) for i in range(a.level + 1)])
        return Ciphertext([c0] + [x.copy() for x in a.c[1:]], a.level, a.scale)


# --------------------------------------------------------------- evaluator
class Evaluator:
    def __init__(self, ctx, u, B, mask=None):
        self.ctx = ctx
        self.T = {1: u}
        self.t1_at = {}
        self.B = B
        self.mask = mask

    def t1_adjusted(self, level, scale):
        key = (level, scale)
        if key not in self.t1_at:
            t1 = self.T[1]
            assert t1.level > level, "level budget exhausted"
            self.t1_at[key] = mul_const(self.ctx, drop(self.ctx, t1, level + 1), 1.0, scale)
        return self.t1_at[key]

    def build(self, j):
        if j in self.T:
            return
        ctx = self.ctx
        if j % 2 == 0:
            self.build(j // 2)
            s = mult(ctx, self.T[j // 2], self.T[j // 2])
            s = scale_int(ctx, s, 2)
            s = add_const(ctx, s, -1.0)
        else:
            self.build((j + 1) // 2)
            self.build((j - 1) // 2)
            s = mult(ctx, self.T[(j + 1) // 2], self.T[(j - 1) // 2])
            s = scale_int(ctx, s, 2)
            s = ctx.sub_ct(s, self.t1_adjusted(s.level, s.scale))
        self.T[j] = s

    def leaf(self, coef, S, lv):
        ctx = self.ctx
        deg = len(coef) - 1
        while deg > 0 and coef[deg] == 0:
            deg -= 1
        if deg == 0:
            return ("const", complex(coef[0]) if coef else 0j)
        ql = float(ctx.q[lv + 1])
        parts = [None, None]
        for j in range(1, deg + 1):
            if coef[j] == 0:
                continue
            self.build(j)
            tj = self.T[j]
            assert tj.level >= lv + 1, "level budget exhausted"
            tjd = drop(ctx, tj, lv + 1)
            for part in (0, 1):
                value = coef[j].real if part == 0 else coef[j].imag
                if value == 0.0:
                    continue
                if self.mask is not None:
                    assert part == 0
                    pscale = S * ql / tj.scale
                    pt = self.mask.plaintext(value * pscale, lv + 1)
                    term = ctx.mul_plain(tjd, pt, 1.0)
                else:
                    K = float(np.rint(value * S * ql / tj.scale))
                    if K == 0.0:
                        continue
                    term = ctx.mul_int(tjd, int(K))
                term.scale = S * ql
                parts[part] = term if parts[part] is None else ctx.add_ct(parts[part], term)
        acc = None
        for part in (0, 1):
            p = parts[part]
            if p is None:
                continue
            if part == 1:
                p = ctx.mul_monomial(p, ctx.N // 2)
            acc = p if acc is None else ctx.add_ct(acc, p)
        if acc is None:
            z = [np.zeros((lv + 2, ctx.N), dtype=np.uint64) for _ in range(2)]
            acc = Ciphertext(z, lv + 1, S * ql)
        c0 = complex(coef[0])
        assert c0.imag == 0.0
        acc = self.mask.add(acc, c0.real) if self.mask is not None else add_const(ctx, acc, c0.real)
        out = ctx.rescale(acc)
        out.scale = S
        return ("ct", out)

    def mul_const_complex(self, g, cv, S):
        ctx = self.ctx
        r = None
        if cv.real != 0.0:
            r = mul_const(ctx, g, cv.real, S)
        if cv.imag != 0.0:
            t = ctx.mul_monomial(mul_const(ctx, g, cv.imag, S), ctx.N // 2)
            r = t if r is None else ctx.add_ct(r, t)
        assert r is not None
        return r

    def eval(self, coef, S, lv):
        ctx = self.ctx
        deg = len(coef) - 1
        while deg > 0 and coef[deg] == 0:
            deg -= 1
        if deg < self.B:
            return self.leaf(coef[:deg + 1], S, lv)
        n = self.B
        while 2 * n <= deg:
            n *= 2
        hi = [coef[n]] + [2.0 * coef[n + k] for k in range(1, deg - n + 1)]
        lo = list(coef[:n])
        for k in range(1, deg - n + 1):
            lo[n - k] -= coef[n + k]
        self.build(n)
        G = self.T[n]
        assert G.level >= lv + 1, "level budget exhausted"
        ql = float(ctx.q[lv + 1])
        vh = self.eval(hi, S * ql / G.scale, lv + 1)
        g = drop(ctx, G, lv + 1)
        if vh[0] == "const" and self.mask is not None:
            assert vh[1].imag == 0.0
            pscale = S * ql / g.scale
            out = ctx.rescale(ctx.mul_plain(g, self.mask.plaintext(vh[1].real * pscale, g.level), pscale))
            out.scale = S
        elif vh[0] == "const":
            out = self.mul_const_complex(g, vh[1], S)
        else:
            out = ctx.rescale(ctx.relinearize(ctx.tensor(vh[1], g)))
            out.scale = S
        vl = self.eval(lo, S, lv)
        if vl[0] == "const":
            assert vl[1].imag == 0.0
            out = self.mask.add(out, vl[1].real) if self.mask is not None else add_const(ctx, out, vl[1].real)
        else:
            out = ctx.add_ct(out, vl[1])
        return ("ct", out)


def eval_cheb(ctx, x, coef, a, b, target_scale, log_scale, mask=None):
    """p(x) = sum_j coef[j] T_j((2x - a - b)/(b - a)) on every slot of x,
    at target_scale; with `mask` (a Mask) the result is p(x) * mu."""
    d = len(coef) - 1
    assert d >= 1
    alpha = 2.0 / (b - a)
    beta = -(a + b) / (b - a)
    fa, ea = math.frexp(alpha)
    if fa == 0.5 and ea >= 1:
        u = scale_int(ctx, x, 1 << (ea - 1))
    else:
        assert x.level >= 1, "level budget exhausted"
        u = mul_const(ctx, x, alpha, float(2 ** log_scale))
    u = add_const(ctx, u, beta)
    t = ceil_log2(d + 1)
    out_level = u.level - (t + 1)
    assert out_level >= 0, "level budget exhausted"
    ev = Evaluator(ctx, u, 1 << max(1, (t + 1) // 2), mask)
    kind, v = ev.eval([complex(c) for c in coef], target_scale, out_level)
    assert kind == "ct"
    return v


def eval_cheb_complex(ctx, x, coef_re, coef_im, target_scale):
    """re(x) + i im(x) for two Chebyshev series on [-1, 1] (x already the
    argument u), one polynomial with complex coefficients."""
    n = max(len(coef_re), len(coef_im))
    coef = [complex(coef_re[j] if j < len(coef_re) else 0.0, coef_im[j] if j < len(coef_im) else 0.0)
            for j in range(n)]
    t = ceil_log2(n)
    out_level = x.level - (t + 1)
    assert out_level >= 0, "level budget exhausted"
    ev = Evaluator(ctx, x, 1 << max(1, (t + 1) // 2))
    kind, v = ev.eval(coef, target_scale, out_level)
    assert kind == "ct"
    return v
