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
* the normalisation polynomial of iteration j is the weighted minimax
  approximant of s^(-e) (polyeval.minimax_invpow; with approx = 1 the
  Chebyshev interpolant instead; e = 1/2, or 2^-j for the
  non-final steps of version B) on [a, a + 2^w] covering the
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


def power_k(n, M, t):
    """Iterations of the normalize-and-t-th-power variant (the appendix on
    other normalisations): M / t^k ~ ln n; t = 2 is the Theorem's k."""
    if t == 2:
        return theorem_k(n, M)
    v = math.ceil((math.log2(M) - math.log2(math.log(float(n)))) / math.log2(float(t)))
    return max(1, int(v))


def power_of(ctx, y, t):
    """y^t, t in {2, 3, 4}: y^2 = y y, then y^2 y or y^2 y^2."""
    y2 = P.mult(ctx, y, y)
    if t == 2:
        return y2
    return P.mult(ctx, y2, y if t == 3 else y2)


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


def default_degree(n, j, last, t=2):
    if t != 2:
        d = (7 if last else 6) if n <= 16 else 7
    elif n <= 256:
        d = 6 if j == 1 else (7 if last else 5)
    elif n <= 1024:
        d = 8 if last else 6
    else:
        d = 8 if last else 7
    return (1 << d) - 1


def newton_delta(delta, steps):
    """Newton's error map for the inverse square root: y sqrt(s) = 1 + e
    becomes 1 - e^2 (3 + e) / 2, so a bound delta becomes delta^2 (3 + delta) / 2."""
    for _ in range(steps):
        delta = delta * delta * (3.0 + delta) / 2.0
    return delta


def newton_invsqrt(ctx, S, y, steps, mask=None, avg=1, tgt=None):
    """Newton's inverse square root iteration (Appendix A, the lemma on
    computing inverse square roots) from the first guess y ~ S^(-1/2):
    y <- 3/2 y - (S/2 y)(y y), two levels per step, each step landing at
    scale tgt exactly: S/2 by a constant product at the scale T1 that puts
    (S/2 y)(y y) at tgt, 3/2 y by a constant product at tgt.  The last step
    also applies the mask (S/2 and 3/2 y as masked plaintext products) or,
    with avg > 1, the averaging factor 1/avg (in both constants); S has levels
    above y, so S/2 costs none of y's."""
    for i in range(steps):
        lastn = i + 1 == steps
        l = y.level
        assert l >= 2 and S.level > l, "Newton step: levels"
        ql, ql1 = float(ctx.q[l]), float(ctx.q[l - 1])
        T1 = tgt * ql * ql * ql1 / (y.scale * y.scale * y.scale)
        if lastn and mask is not None:
            qs = float(ctx.q[S.level])
            ps = T1 * qs / S.scale
            h = ctx.rescale(ctx.mul_plain(S, mask.plaintext(0.5 * ps, S.level), ps))
            h.scale = T1
        else:
            h = P.mul_const(ctx, S, 0.5 / avg if lastn else 0.5, T1)
        z1 = P.mult(ctx, h, y)
        z2 = P.mult(ctx, y, y)
        w = P.mult(ctx, z1, z2)
        if lastn and mask is not None:
            ps = tgt * ql / y.scale
            z3 = ctx.rescale(ctx.mul_plain(y, mask.plaintext(1.5 * ps, l), ps))
            z3.scale = tgt
        else:
            z3 = P.mul_const(ctx, y, 1.5 / avg if lastn else 1.5, tgt)
        y = ctx.sub_ct(P.drop(ctx, z3, w.level), w)
    return y


def softmax(ctx, xs, n, M, variant=0, k=0, exp_degree=15, inv_degrees=(0, 0, 0), bootstrap=None,
            debug_stop=-1, stats=None, power=2, newton_steps=0, mask_mode=0, approx=0, boot_top=None, jobs=1,
            merge=False):
    """Softmax of the L = m N0 / n2 vectors packed in the oracle ciphertexts
    xs (m of them, one level and scale, inputs in [-M, 0]); n2 is n rounded
    up to a power of two (the packing's dimension; the extra coordinates are
    masked out after the exponential).  power: normalize-and-t-th-power (the
    appendix on other normalisations; 2 is normalize-and-square).
    Returns the m output ciphertexts.  The context must hold the
    relinearisation key; the rotation keys of strides +-L 2^t are added
    here.  newton_steps > 0: each inverse square root is the polynomial's
    first guess refined by that many Newton steps (squares only; version B
    takes an inverse square root in its last step only); 0: by dimension,
    none up to n = 2048 and two above; -1: none.  mask_mode 1: the averaging mask, the factor divided by n2/m on
    every slot instead of the indicator of slots [0, L).

    jobs > 1 with merge (version B only): xs holds `jobs` consecutive jobs of
    len(xs) / jobs ciphertexts, whose auxiliary ciphertexts are packed (Section
    4.2: one auxiliary ciphertext carries the sums of many Softmax), Jg =
    min(jobs, n2 / m) jobs per ciphertext: after each job's rotate-and-add,
    job g Jg + b's sums (on every block of L slots) keep block b by a 0/1
    plaintext of that block at scale q_l, summed over the group's jobs before
    one rescale; the polynomials and bootstraps act on the packed ciphertexts
    (indicator of slots [0, Jg L)); a factor is taken apart the same way (job
    g Jg + b: block b's plaintext on the g-th, one rescale) and broadcast.
    Every y^(j) then keeps two levels (one for the packing)."""
    N0 = ctx.slots
    J = jobs
    m = len(xs) // J
    assert J >= 1 and J * m == len(xs)
    assert J == 1 or merge, "lockstep jobs without packing equal the jobs run one by one"
    mg = bool(merge) and J > 1
    n2 = 1 << ilog2(n)
    assert n >= 2 and n2 <= N0 and n2 % m == 0
    tp = power
    assert tp in (2, 3, 4) and (tp == 2 or variant == 0)
    assert newton_steps <= 0 or tp == 2
    if newton_steps == 0:
        newton_steps = 2 if (tp == 2 and n > 2048) else 0
    newton_opt = max(newton_steps, 0)
    avg = mask_mode == 1
    tl = 1 if tp == 2 else 2         # levels of y^tp
    L = m * N0 // n2
    k = k if k > 0 else power_k(n, M, tp) + (1 if n >= 4096 else 0)
    per = n2 // m
    nrot = ilog2(per)
    smb = variant == 1
    assert not merge or (smb and mask_mode == 0 and newton_opt == 0 and (J <= per or J % per == 0))
    Jg = min(J, per)
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

    # v = 2x / M in [-2, 0]: a declared-scale change; one rescale first for
    # inputs encrypted at (2 Delta / M) q_l (the encryption noise divided by
    # q_l); otherwise a constant product
    vs = xs[0].scale * M / 2.0
    lx = xs[0].level
    if abs(math.log2(vs) - log_scale) <= 2.0:
        v = []
        for x in xs:
            c = x.copy()
            c.scale = vs
            v.append(c)
    elif lx >= 1 and abs(math.log2(vs / float(ctx.q[lx])) - log_scale) <= 2.0:
        v = []
        for x in xs:
            c = ctx.rescale(x)
            c.scale = c.scale * M / 2.0
            v.append(c)
    else:
        v = [P.mul_const(ctx, x, 2.0 / M, Delta) for x in xs]
    # y0 = exp(x / tp^k) / n^(1/tp): sum y0^tp in [e^(-tp M / tp^k), 1]
    isn = 1.0 / math.sqrt(n) if tp == 2 else math.pow(float(n), -1.0 / tp)
    Mm, kk = mpmath.mpf(M), k
    tk2 = mpmath.mpf(2) ** (kk + 1) if tp == 2 else 2 * mpmath.mpf(tp) ** kk
    pexp = P.cheb_interp(lambda u: mpmath.exp(Mm * u / tk2) * mpmath.mpf(isn), -2.0, 0.0, exp_degree)
    y0 = [P.eval_cheb(ctx, c, pexp, -2.0, 0.0, Delta, log_scale) for c in v]
    if n2 != n:
        # padded dimension: ciphertext j keeps slots [0, R_j), R_j = (n - j
        # per) L in [0, N0] (its real coordinates), by a 0/1 plaintext at
        # scale q_l and one rescale; the scale stays y0's
        out = []
        for j, c in enumerate(y0):
            R = min(max((n - j * per) * L, 0), N0)
            ql = float(ctx.q[c.level])
            pt = P.Mask(ctx, [1.0] * R + [0.0] * (N0 - R)).plaintext(ql, c.level)
            r = ctx.rescale(ctx.mul_plain(c, pt, ql))
            r.scale = c.scale
            out.append(r)
        y0 = out
    if debug_stop == 0:
        return y0
    LM = Jg * L if mg else L
    mask = P.Mask(ctx, [1.0] * LM + [0.0] * (N0 - LM))
    blocks = [P.Mask(ctx, [0.0] * (b * L) + [1.0] * L + [0.0] * (N0 - (b + 1) * L)) for b in range(Jg)] if mg else []

    def pack(Ss):
        # job g Jg + b keeps block b of the g-th: sums of S_i times block
        # plaintexts at q_l, one rescale
        lvl = Ss[0].level
        assert lvl >= 1, "no level to pack the jobs' auxiliary ciphertexts"
        ql = float(ctx.q[lvl])
        out = []
        for g in range(J // Jg):
            acc = None
            for b in range(Jg):
                t_ = ctx.mul_plain(Ss[g * Jg + b], blocks[b].plaintext(ql, lvl), ql)
                acc = t_ if acc is None else ctx.add_ct(acc, t_)
            r_ = ctx.rescale(acc)
            r_.scale = Ss[0].scale
            out.append(r_)
        return out

    def unpack(As):
        # job g Jg + b's factor: A_g times block b's plaintext at q_l, one rescale
        lvl = As[0].level
        assert lvl >= 1, "no level to take the jobs' factors apart"
        ql = float(ctx.q[lvl])
        out = []
        for i in range(J):
            r_ = ctx.rescale(ctx.mul_plain(As[i // Jg], blocks[i % Jg].plaintext(ql, lvl), ql))
            r_.scale = As[0].scale
            out.append(r_)
        return out

    y = list(y0)
    big = None
    ybound = isn * 1.05
    lo = (math.exp(-2.0 * M / math.ldexp(1.0, k)) if tp == 2 else math.exp(-tp * M / math.pow(float(tp), k))) * 0.98
    hi = 1.0
    for j in range(1, k + 1):
        last = j == k
        smb_step = smb and not last
        # Newton's steps on the inverse square roots only (version B: its last step)
        newton_steps = 0 if smb_step else newton_opt
        e = math.ldexp(1.0, -j) if smb_step else (0.5 if tp == 2 else 1.0 / tp)
        deg = inv_degrees[0] if j == 1 else (inv_degrees[2] if last else inv_degrees[1])
        if deg <= 0:
            deg = default_degree(n, j, last, tp)
        if not smb:
            y = [ensure(c, 1 + tl if last else 1 + 2 * tl, ybound) for c in y]
        # auxiliary thread: S = sum of the t-th powers (squares: the tensors
        # summed, one relinearisation), rotate-and-add; per job, then packed
        Ss = []
        for i in range(J):
            yj = y[i * m:(i + 1) * m]
            if tp == 2:
                d = ctx.tensor(yj[0], yj[0])
                for c in yj[1:]:
                    d = ctx.add_ct(d, ctx.tensor(c, c))
                S = ctx.rescale(ctx.relinearize(d))
            else:
                yt = [power_of(ctx, c, tp) for c in yj]
                S = yt[0]
                for c in yt[1:]:
                    S = ctx.add_ct(S, c)
            for t in range(nrot):
                S = ctx.add_ct(S, ctx.rotate(S, -(L << t)))
            Ss.append(S)
        # the auxiliary ciphertexts: the packed ones, or the job's own
        Sl = pack(Ss) if mg else [Ss[0]]
        # lambda lands depth (+ 1 when the affine map takes a level) + 2
        # newton_steps below S; the cube and fourth power variants and
        # Newton's steps also keep 1 + tl levels in lambda
        # the last step's z = lambda y and z^2 take two of lambda's levels;
        # packed jobs: one more for taking the factor apart
        keep = (2 + tl if (tp != 2 or newton_steps) else (1 + tl if last else 1)) + (1 if mg and not smb_step else 0)
        # when that exceeds the level a bootstrapping restores (boot_top),
        # Newton's first guess is bootstrapped before the steps
        need_full = P.depth(deg) + 2 * newton_steps + keep
        refresh = newton_steps > 0 and bootstrap is not None and boot_top is not None and need_full > boot_top
        Sl = [ensure(s_, max(P.depth(deg), 2 * newton_steps + keep + 1) if refresh else need_full, hi * 1.1)
              for s_ in Sl]
        S = Sl[0]
        # the polynomial's interval: [lo, lo + 2^w] (integer affine map); in the
        # last step of SM with squares exactly [lo, hi] when S has the level
        # its affine map takes on top of the polynomial and z = lambda y, z^2
        if last and tp == 2 and not newton_steps and S.level >= P.depth(deg) + 3 + (1 if mg else 0):
            a, b = lo, hi
        else:
            a, b = free_interval(lo, hi)
        if approx == 0:
            pinv = P.minimax_invpow(a, b, deg, e)
        else:
            ee = mpmath.mpf(e)
            pinv = P.cheb_interp(lambda s: mpmath.power(s, -ee), a, b, deg)
        delta0 = rel_error(pinv, a, b, lo, hi, e)
        delta = newton_delta(delta0, newton_steps)
        lam_bound = ((1.0 + delta) / math.sqrt(lo) if newton_steps else max_abs(pinv, a, b, lo, hi)) * 1.05
        pe = [cf / per for cf in pinv] if avg and not newton_steps else pinv
        if avg:
            lam_bound /= per
        if not newton_steps:
            laml = [P.eval_cheb(ctx, s_, pe, a, b, Delta, log_scale, None if avg else mask) for s_ in Sl]
        else:
            g = P.eval_cheb(ctx, S, pinv, a, b, Delta, log_scale)
            if refresh:
                g = ensure(g, 2 * newton_steps + keep, (1.0 + delta0) / math.sqrt(lo) * 1.05)
                if g.level >= S.level:
                    g = P.drop(ctx, g, S.level - 1)
            laml = [newton_invsqrt(ctx, S, g, newton_steps, None if avg else mask, per if avg else 1, Delta)]
        if not smb_step:
            need_next = 1 + tl if j + 1 == k else 1 + 2 * tl
            lv_ = laml[0].level
            if not last and bootstrap is not None and lv_ < y[0].level and lv_ - 1 - tl < need_next:
                laml = [ensure(l_, y[0].level, lam_bound, 0 if avg else L) for l_ in laml]
            lams = [broadcast(l_) for l_ in (unpack(laml) if mg else laml)]
            z = [P.mult(ctx, c, lams[i // m]) for i, c in enumerate(y)]
            y = [power_of(ctx, c, tp) for c in z]
            # sum y in [(1 - delta)^tp, (1 + delta)^tp]; by the power-mean
            # inequality sum y^tp in [(1 - delta)^(tp^2) / n^(tp-1), (1 + delta)^(tp^2)]
            if tp == 2:
                lo = math.pow(1.0 - delta, 4.0) / n * 0.98
                hi = math.pow(1.0 + delta, 4.0) * 1.0001
            else:
                lo = math.pow(1.0 - delta, float(tp * tp)) / math.pow(float(n), tp - 1.0) * 0.98
                hi = math.pow(1.0 + delta, float(tp * tp)) * 1.0001
            ybound = hi * 1.05
        else:
            if avg:
                laml = [broadcast(l_) for l_ in laml]
            big = laml if big is None else [P.mult(ctx, b_, l_) for b_, l_ in zip(big, laml)]
            r = 2 if (j == k - 1 or mg) else 1
            want = j + 1 + r
            assert y0[0].level >= want, "version B: main-thread level budget exhausted"
            want_big = want + (1 if mg else 0)
            if big[0].level < want_big:
                big = [ensure(b_, want_big, max(64.0, lam_bound * per if avg else lam_bound, 4.0 * math.sqrt(n)),
                              0 if avg else LM) for b_ in big]
            bbs = unpack(big) if mg else list(big)
            if not avg:
                bbs = [broadcast(b_) for b_ in bbs]
            y = [P.mult(ctx, c, bbs[i // m]) for i, c in enumerate(y0)]
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
