"""CKKS bootstrapping on oracle ciphertexts (coefficient-to-slot first).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper refreshes ciphertexts with its library's bootstrapping and states
only what it is for (Section 2.2, "Levels": a ciphertext whose levels are
spent is brought back to a full budget) and its cost and precision
(Section 5.1).  This module implements the pipeline the HIP library
specifies, step by step, with plain operations: every linear transform is
the diagonal method (one rotation and one plaintext product per nonzero
diagonal, no baby-step giant-step, no hoisting), and its matrices are dense
products of butterfly stages computed here.

 1. Message size: with B = max(bound, 2^-20) and target q0 / 2^9, if
    B scale > 2 target and the level is >= 1, multiply by 2^-e (a constant
    product at the same scale) with e = ceil(log2(B scale / target));
    otherwise multiply by the integer kf = min(floor(target / (B scale)), 16)
    when kf >= 2 (scale times kf).  Keep q0 and lift it to every Q prime
    (ModRaise): t = m + q0 I, declared scale s0 = 2 q0 (K+1) n (n = N/2).
 2. CoeffToSlot: the butterfly stages of the inverse special FFT (lengths
    n, n/2, ..., 2, without its bit reversal and its 1/n), grouped into
    `cts_levels` products (larger groups first), one level each; slot j
    then holds (t_brv(j) + i t_brv(j)+n) / (2 q0 (K+1)).  Level g's
    plaintext scale takes the ciphertext from scale s_g to
    s_(g+1) = 2^((1-f) log2 s0 + f log2 2^log_boot_scale), f = (g+1)/levels;
    the last level is not rescaled.
 3. u_re = t + conj(t), u_im = (t - conj(t)) X^(3N/2) (times -i): 2 Re, 2 Im;
    one rescale each.
 4. EvalMod: z = C(u) + i S(u) with C, S the Chebyshev interpolants of
    cos(w u), sin(w u) on [-1, 1] (degree cos_degree, w = 2 pi (K+1) /
    2^r; the odd terms of C and even terms of S set to 0), as one polynomial
    with complex coefficients at scale D 2^log_boot_scale kf^(-2^-(r+1));
    then r squarings: z = exp(2 pi i t / q0).
 5. V = z (8 - z): Im V = 8 sin x - sin 2x, x = 2 pi t / q0 (no cubic term).
 6. With V_re, V_im the two halves: A = V_re X^(3N/2) + V_im,
    B = V_re X^(N/2) + V_im, v = A - conj(B) = 2 Im V_re + 2i Im V_im.
 7. SlotToCoeff: the forward butterfly stages (lengths 2, ..., n) grouped
    into `stc_levels` products (larger groups last), the factor
    q0 / (24 pi Delta) folded into the first, scales from kf scale(v) to
    Delta = 2^log_scale geometrically; with a mask length L the last
    product's rows L.. are zero (the output is masked to slots [0, L)).
    Output scale: scale(y) s_msg / Delta (s_msg the scale after step 1),
    times the integer 2^e when step 1 divided by 2^e.
"""
import ctypes
import math

import mpmath
import numpy as np

from .encoding import twiddles
from . import polyeval as P


_libm = ctypes.CDLL("libm.so.6")
_libm.exp2.restype = ctypes.c_double
_libm.exp2.argtypes = [ctypes.c_double]


def exp2(x):
    """C's exp2 (the scale plans below use it)."""
    return _libm.exp2(x)


def _stage_exps(N, length):
    h = length // 2
    lq = 4 * length
    e = []
    p = 1
    for _ in range(h):
        e.append(p * (2 * N // lq))
        p = p * 5 % lq
    return e


def stage_matrix(N, length, inverse):
    """Dense n x n matrix of one butterfly stage on blocks of `length`:
    inverse: (a, b) -> (a + b, (a - b) conj(W_j)); forward: (a, b) ->
    (a + W_j b, a - W_j b), W_j = zeta^(e_j), zeta = exp(i pi / N)."""
    n = N // 2
    cos, sin = twiddles(N)
    e = _stage_exps(N, length)
    h = length // 2
    A = np.zeros((n, n), dtype=np.complex128)
    for base in range(0, n, length):
        for j in range(h):
            w = complex(cos[e[j]], sin[e[j]])
            a, b = base + j, base + j + h
            if inverse:
                A[a, a] = 1.0
                A[a, b] = 1.0
                A[b, a] = w.conjugate()
                A[b, b] = -w.conjugate()
            else:
                A[a, a] = 1.0
                A[a, b] = w
                A[b, a] = 1.0
                A[b, b] = -w
    return A


def group_sizes(nst, g):
    s = [nst // g] * g
    for i in range(nst % g):
        s[i] += 1
    return s


def diagonals(M):
    """{d: diag_d} with M x = sum_d diag_d * rot(x, d) (left rotations)."""
    n = M.shape[0]
    out = {}
    idx = np.arange(n)
    for d in range(n):
        v = M[idx, (idx + d) % n]
        if np.any(v != 0):
            out[d] = v
    return out


class Bootstrapper:
    def __init__(self, ctx, boot, user_top, log_scale):
        self.ctx = ctx
        self.bp = dict(boot)
        self.user_top = user_top
        self.log_scale = log_scale
        N = ctx.N
        n = N // 2
        nst = n.bit_length() - 1
        bp = self.bp
        # CoeffToSlot factors: stages n, n/2, ..., 2 in application order
        self.cts = []
        length = n
        for gsz in group_sizes(nst, bp["cts_levels"]):
            M = np.eye(n, dtype=np.complex128)
            for _ in range(gsz):
                M = stage_matrix(N, length, True) @ M
                length //= 2
            self.cts.append(diagonals(M))
        # SlotToCoeff factors: stages 2, 4, ..., n
        self.stc = []
        length = 2
        for gsz in reversed(group_sizes(nst, bp["stc_levels"])):
            M = np.eye(n, dtype=np.complex128)
            for _ in range(gsz):
                M = stage_matrix(N, length, False) @ M
                length *= 2
            self.stc.append(M)
        K, r = bp["K"], bp["double_angle"]
        w = 2 * mpmath.pi * (K + 1) / mpmath.mpf(2) ** r
        self.pcos = P.cheb_interp(lambda u: mpmath.cos(w * u), -1.0, 1.0, bp["cos_degree"])
        self.psin = P.cheb_interp(lambda u: mpmath.sin(w * u), -1.0, 1.0, bp["cos_degree"])
        for j in range(len(self.pcos)):
            if j % 2:
                self.pcos[j] = 0.0
            else:
                self.psin[j] = 0.0
        self.keys_done = False

    def rotations(self):
        rs = set()
        for D in self.cts:
            rs |= set(D)
        for M in self.stc:
            rs |= set(diagonals(M))
        return sorted(r for r in rs if r)

    def _keys(self):
        if self.keys_done:
            return
        ctx = self.ctx
        ctx.add_galois_key(2 * ctx.N - 1)
        for r in self.rotations():
            ctx.add_galois_key(ctx.galois_rot(r, ctx.N))
        self.keys_done = True

    def _linear(self, x, D, pt_scale, rescale=True):
        """sum_d diag_d * rot(x, d), plaintexts at pt_scale, one rescale."""
        ctx = self.ctx
        acc = None
        for d, v in D.items():
            xr = x if d == 0 else ctx.rotate(x, d)
            pt, _ = ctx.encode(v, pt_scale, x.level)
            t = ctx.mul_plain(xr, pt, pt_scale)
            acc = t if acc is None else ctx.add_ct(acc, t)
        return ctx.rescale(acc) if rescale else acc

    def bootstrap(self, x, bound=1.0, mask_L=0, stop=0, trace=None):
        """Refresh x (any level) to level user_top.  stop > 0 returns an
        intermediate ciphertext (the numbering of the library's test hook):
        1 after ModRaise, 2 after CoeffToSlot (rescaled), 3 u_re, 4 the real
        half of z after the polynomial, 5 / 6 the real / imaginary half of z
        after the squarings, 7 the SlotToCoeff input, 8 / 9 after its first
        / second level.  A dict `trace` receives every one of them."""
        def mark(k, c):
            if trace is not None:
                trace[k] = c
            return stop == k

        ctx = self.ctx
        bp = self.bp
        self._keys()
        N = ctx.N
        n = N // 2
        q0 = float(ctx.q[0])
        L = ctx.L
        Db = math.ldexp(1.0, bp["log_boot_scale"])
        Bd = max(bound, math.ldexp(1.0, -20))
        # 1. message size
        target = q0 / 512.0
        e = 0
        kfac = 1.0
        if Bd * x.scale > 2.0 * target and x.level >= 1:
            e = int(math.ceil(math.log2(Bd * x.scale / target)))
            xx = P.mul_const(ctx, x, math.ldexp(1.0, -e), x.scale)
        else:
            xx = x.copy()
            kf = min(math.floor(target / (Bd * x.scale)), 16.0)
            if kf >= 2.0:
                xx = ctx.mul_int(xx, int(kf))
                xx.scale = x.scale * float(int(kf))
                kfac = float(int(kf))
        s_msg = xx.scale
        t = ctx.mod_raise(ctx.mod_drop(xx, 0), L)
        s0 = 2.0 * q0 * (bp["K"] + 1) * n
        t.scale = s0
        if mark(1, t):
            return t
        # 2. CoeffToSlot
        s_prev = s0
        ncts = len(self.cts)
        for gi, D in enumerate(self.cts):
            frac = (gi + 1) / ncts
            s_next = exp2(math.log2(s0) * (1 - frac) + math.log2(Db) * frac)
            lvl = L - gi
            assert t.level == lvl
            pt_scale = s_next * float(ctx.q[lvl]) / s_prev
            t = self._linear(t, D, pt_scale, rescale=gi + 1 < ncts)
            s_prev = s_prev * pt_scale / float(ctx.q[lvl])
        if stop == 2 or trace is not None:
            t2 = ctx.rescale(t)
            if mark(2, t2):
                return t2
        # 3. real / imaginary split
        cj = ctx.conjugate(t)
        ure = ctx.rescale(ctx.add_ct(t, cj))
        uim = ctx.rescale(ctx.mul_monomial(ctx.sub_ct(t, cj), 3 * N // 2))
        if mark(3, ure):
            return ure
        # 4. EvalMod
        r = bp["double_angle"]
        Dp = Db * math.pow(kfac, -math.ldexp(1.0, -(r + 1)))
        z = [P.eval_cheb_complex(ctx, u, self.pcos, self.psin, Dp) for u in (ure, uim)]
        if mark(4, z[0]):
            return z[0]
        for _ in range(r):
            z = [ctx.mult(c, c) for c in z]
        if mark(5, z[0]) or mark(6, z[1]):
            return z[stop - 5]
        # 5. V = z (8 - z)
        V = []
        for c in z:
            w8 = P.add_const(ctx, ctx.mul_int(c, -1), 8.0)
            V.append(ctx.mult(c, w8))
        # 6. v = 2 Im V_re + 2i Im V_im
        A = ctx.add_ct(ctx.mul_monomial(V[0], 3 * N // 2), V[1])
        B = ctx.add_ct(ctx.mul_monomial(V[0], N // 2), V[1])
        y = ctx.sub_ct(A, ctx.conjugate(B))
        if mark(7, y):
            return y
        # 7. SlotToCoeff
        Dout = math.ldexp(1.0, self.log_scale)
        cst = q0 / (12.0 * 6.283185307179586 * Dout)
        in_scale = y.scale * kfac
        s_prev = in_scale
        nstc = len(self.stc)
        for gi, M in enumerate(self.stc):
            frac = (gi + 1) / nstc
            s_next = exp2(math.log2(in_scale) * (1 - frac) + math.log2(Dout) * frac)
            lvl = self.user_top + nstc - gi
            assert y.level == lvl
            pt_scale = s_next * float(ctx.q[lvl]) / s_prev
            Mg = M * cst if gi == 0 else M.copy()
            if mask_L > 0 and gi + 1 == nstc:
                Mg[mask_L:, :] = 0.0
            y = self._linear(y, diagonals(Mg), pt_scale)
            s_prev = s_prev * pt_scale / float(ctx.q[lvl])
            if gi + 1 < nstc and mark(8 + gi, y):
                return y
        y.scale = y.scale * s_msg / Dout
        if e > 0:
            y = ctx.mul_int(y, 1 << e)
        return y
