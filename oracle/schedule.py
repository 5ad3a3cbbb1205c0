"""The encrypted Softmax schedule on oracle ciphertexts: Algorithm SM and
SM version B with the auxiliary thread and the many-ciphertext packing.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Steps, in the paper's order and notation:

* Algorithm SM (Section 3.2): y0 = exp(x / 2^k); for j = 1..k:
  lambda = (sum_i y_i^2)^(-1/2) from the auxiliary thread, z = lambda y,
  y = z^2.
* The auxiliary thread (Algorithm "alg:AuxThread", Section 3.3) on m packed
  ciphertexts (Section 4.2): the squares of the m ciphertexts summed (one
  relinearisation), rotate-and-add with strides -L 2^t for t < log2(n/m),
  the normalisation polynomial with the mask of slots [0, L) folded into its
  constants, rotate-and-add with strides +L 2^t.
* Version B (Algorithm "alg:Softmax1B", Section 4.3): lambda_j =
  (sum y^(j-1)^2)^(-2^-j), Lambda = Lambda lambda_j, z = Lambda y0,
  y^(j) = z^(2^j); its last iteration is one normalize-and-square step on
  y^(k-1) (the same value y^(k-1)^2 / S_k with an error not amplified 2^k).

Readings where the paper leaves a choice (the HIP library makes the same):
* k = ceil(log2 M - log2 ln n) (Theorem "th:prec_softmax"), plus one from
  n = 4096 on;
* y0 is prescaled by 1/sqrt(n) (exp(M t / 2^(k+1)) / sqrt(n) on t = 2x/M in
  [-2, 0], degree 15 by default) so sum y0^2 lies in [e^(-2M/2^k), 1];
* the normalisation polynomial of iteration j interpolates s^(-e) (e = 1/2,
  or 2^-j for the non-final steps of version B) on [a, a + 2^w] covering the
  interval [lo, hi] that the previous step's measured relative error gives
  (Section 5.1: [(1 - alpha)^2 / n, (1 + alpha)^2], with margins); degrees
  2^d - 1 with d from the paper's level table of the auxiliary thread;
* bootstraps: the main ciphertexts when their levels run out (SM), the
  auxiliary ciphertext before the polynomial when its budget is short, and
  the normalisation factors on slots [0, L) before their broadcast, with the
  mask applied by the bootstrap (Section 5.1, bootstrapping strategy).  The
  bootstrap is passed in (``bootstrap(ct, bound, mask_L)``); without one a
  short budget is an error.
"""
import math

import mpmath

from . import polyeval as P


def theorem_k(n, M):
    v = math.ceil(math.log2(M) - math.log2(math.log(float(n))))
    return max(1, int(v))


def ilog2(x):
    l = 0
    while (1 << l) < x:
        l += 1
    return l


def rel_error(coef, a, b, lo, hi, e):
    """max over a geometric grid of [lo, hi] of |p(s) s^e - 1| (double)."""
    worst = 0.0
    G = 4000
    for i in range(G + 1):
        s = lo * math.pow(hi / lo, i / G)
        worst = max(worst, abs(P.cheb_eval_plain(coef, a, b, s) * math.pow(s, e) - 1.0))
    return worst


def max_abs(coef, a, b, lo, hi):
    m = 0.0
    for i in range(2001):
        m = max(m, abs(P.cheb_eval_plain(coef, a, b, lo + (hi - lo) * i / 2000.0)))
    return m


def free_interval(lo, hi):
    """[a, a + 2^w] covering [lo, hi] with 2^w <= 2 (2^w >= 1/64)."""
    w = 1.0
    while w < hi - lo:
        w *= 2
    while w / 2 >= hi - lo and w > 1.0 / 64:
        w /= 2
    return lo, lo + w


def default_degree(n, j, last):
    if n <= 256:
        d = 6 if j == 1 else (7 if last else 5)
    elif n <= 1024:
        d = 8 if last else 6
    else:
        d = 8 if last else 7
    return (1 << d) - 1


def softmax(ctx, xs, n, M, variant=0, k=0, exp_degree=15, inv_degrees=(0, 0, 0), bootstrap=None,
            debug_stop=-1, stats=None):
    """Softmax of the L = m N0 / n vectors packed in the oracle ciphertexts
    xs (m of them, one level and scale, inputs in [-M, 0]); returns the m
    output ciphertexts.  The context must hold the relinearisation key; the
    rotation keys of strides +-L 2^t are added here."""
    N0 = ctx.slots
    m = len(xs)
    assert n >= 2 and n & (n - 1) == 0 and n <= N0 and n % m == 0
    L = m * N0 // n
    k = k if k > 0 else theorem_k(n, M) + (1 if n >= 4096 else 0)
    nrot = ilog2(n // m)
    smb = variant == 1
    log_scale = int(round(math.log2(ctx.delta)))
    Delta = math.ldexp(1.0, log_scale)
    for t in range(nrot):
        ctx.add_galois_key(ctx.galois_rot(-(L << t), ctx.N))
        ctx.add_galois_key(ctx.galois_rot(L << t, ctx.N))
    st = dict(k=k, bootstraps=0)

    def ensure(x, need, bound, mask_L=0):
        if x.level >= need:
            return x
        assert bootstrap is not None, "level budget exhausted and no bootstrapping"
        st["bootstraps"] += 1
        out = bootstrap(x, bound, mask_L)
        assert out.level >= need
        return out

    def broadcast(a):
        for t in range(nrot):
            a = ctx.add_ct(a, ctx.rotate(a, L << t))
        return a

    # v = 2x / M in [-2, 0]: a declared-scale change, or a constant product
    vs = xs[0].scale * M / 2.0
    if abs(math.log2(vs) - log_scale) <= 2.0:
        v = []
        for x in xs:
            c = x.copy()
            c.scale = vs
            v.append(c)
    else:
        v = [P.mul_const(ctx, x, 2.0 / M, Delta) for x in xs]
    isn = 1.0 / math.sqrt(n)
    Mm, kk = mpmath.mpf(M), k
    pexp = P.cheb_interp(lambda t: mpmath.exp(Mm * t / mpmath.mpf(2) ** (kk + 1)) * mpmath.mpf(isn),
                         -2.0, 0.0, exp_degree)
    y0 = [P.eval_cheb(ctx, c, pexp, -2.0, 0.0, Delta, log_scale) for c in v]
    if debug_stop == 0:
        return y0
    mask = P.Mask(ctx, [1.0] * L + [0.0] * (N0 - L))

    y = list(y0)
    big = None
    ybound = isn * 1.05
    lo = math.exp(-2.0 * M / math.ldexp(1.0, k)) * 0.98
    hi = 1.0
    for j in range(1, k + 1):
        last = j == k
        smb_step = smb and not last
        e = math.ldexp(1.0, -j) if smb_step else 0.5
        deg = inv_degrees[0] if j == 1 else (inv_degrees[2] if last else inv_degrees[1])
        if deg <= 0:
            deg = default_degree(n, j, last)
        a, b = free_interval(lo, hi)
        ee = mpmath.mpf(e)
        pinv = P.cheb_interp(lambda s: mpmath.power(s, -ee), a, b, deg)
        delta = rel_error(pinv, a, b, lo, hi, e)
        lam_bound = max_abs(pinv, a, b, lo, hi) * 1.05
        if not smb:
            y = [ensure(c, 2 if last else 3, ybound) for c in y]
        # auxiliary thread: S = sum of the squares, rotate-and-add
        d = ctx.tensor(y[0], y[0])
        for c in y[1:]:
            d = ctx.add_ct(d, ctx.tensor(c, c))
        S = ctx.rescale(ctx.relinearize(d))
        for t in range(nrot):
            S = ctx.add_ct(S, ctx.rotate(S, -(L << t)))
        S = ensure(S, P.depth(deg) + 1, hi * 1.1)
        lam = P.eval_cheb(ctx, S, pinv, a, b, Delta, log_scale, mask)
        if not smb_step:
            need_next = 2 if j + 1 == k else 3
            if not last and bootstrap is not None and lam.level < y[0].level and lam.level - 2 < need_next:
                lam = ensure(lam, y[0].level, lam_bound, L)
            lam = broadcast(lam)
            z = [P.mult(ctx, c, lam) for c in y]
            y = [P.mult(ctx, c, c) for c in z]
            lo = math.pow(1.0 - delta, 4.0) / n * 0.98
            hi = math.pow(1.0 + delta, 4.0) * 1.0001
            ybound = hi * 1.05
        else:
            big = lam if big is None else P.mult(ctx, big, lam)
            r = 2 if j == k - 1 else 1
            want = j + 1 + r
            assert y0[0].level >= want, "version B: main-thread level budget exhausted"
            if big.level < want:
                big = ensure(big, want, max(64.0, lam_bound, 4.0 * math.sqrt(n)), L)
            bb = broadcast(big)
            y = [P.mult(ctx, c, bb) for c in y0]
            for _ in range(j):
                y = [P.mult(ctx, c, c) for c in y]
            ej = math.ldexp(1.0, j + 1)
            lo = math.pow(1.0 - delta, ej) / n * 0.98
            hi = math.pow(1.0 + delta, ej) * 1.0001
        if debug_stop == j:
            break
    if stats is not None:
        stats.update(st)
    return y
