"""Polynomial approximations used by the method (Section 5.1, "Designing
auxiliary functions"; Appendix A).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper computes minimax approximants with Sollya: for the exponential a
plain minimax fit, for x^(-1/2) a weighted fit minimising max |P(x) sqrt(x) - 1|,
with degrees 2^t - 1.  Sollya is not available here; this module gives

* ``cheb_interp``: interpolation at the d+1 Chebyshev nodes of the first kind
  (coefficients in the Chebyshev basis of the interval), and
* ``remez``: the Remez exchange for the weighted problem
  min_P max_x |w(x) (P(x) - f(x))| in the Chebyshev basis,

and the interval rules of Section 5.1: after a normalisation with
|lambda^2 sum y^2 - 1| <= alpha, the next input lies in
[(1 - alpha)^2 / n, (1 + alpha)^2].
"""
import numpy as np
from numpy.polynomial import chebyshev as C


def to_unit(x, a, b):
    return (2.0 * np.asarray(x, dtype=np.float64) - a - b) / (b - a)


def cheb_eval(coef, x, a, b):
    return C.chebval(to_unit(x, a, b), coef)


def cheb_interp(f, a, b, d):
    """Coefficients c_0..c_d with sum c_j T_j(u) interpolating f at the
    Chebyshev nodes u_k = cos(pi (k + 1/2) / (d + 1))."""
    k = np.arange(d + 1)
    u = np.cos(np.pi * (k + 0.5) / (d + 1))
    x = (u * (b - a) + a + b) / 2.0
    fx = f(x)
    c = np.empty(d + 1)
    for j in range(d + 1):
        c[j] = 2.0 / (d + 1) * np.sum(fx * np.cos(np.pi * j * (k + 0.5) / (d + 1)))
    c[0] /= 2.0
    return c


def remez(f, w, a, b, d, iters=60, grid=20001, tol=1e-12):
    """Weighted minimax approximation of f on [a, b] by a degree-d
    polynomial: minimise max |w(x) (P(x) - f(x))|.  Returns (coef, err)."""
    # initial reference: Chebyshev extrema
    k = np.arange(d + 2)
    u_ref = -np.cos(np.pi * k / (d + 1))
    gu = np.cos(np.pi * (np.arange(grid) + 0.5) / grid)[::-1]
    gu = np.concatenate([[-1.0], gu, [1.0]])
    gx = (gu * (b - a) + a + b) / 2.0
    fg = f(gx)
    wg = w(gx)
    err = None
    coef = None
    for _ in range(iters):
        xr = (u_ref * (b - a) + a + b) / 2.0
        A = np.zeros((d + 2, d + 2))
        for j in range(d + 1):
            e = np.zeros(j + 1)
            e[j] = 1.0
            A[:, j] = C.chebval(u_ref, e)
        A[:, d + 1] = ((-1.0) ** k) / w(xr)
        sol = np.linalg.solve(A, f(xr))
        coef = sol[:d + 1]
        E = wg * (C.chebval(gu, coef) - fg)
        # new reference: one extremum per sign-alternating run
        sign = np.sign(E)
        sign[sign == 0] = 1
        idx = []
        start = 0
        for i in range(1, len(E) + 1):
            if i == len(E) or sign[i] != sign[start]:
                seg = np.arange(start, i)
                idx.append(seg[np.argmax(np.abs(E[seg]))])
                start = i
        idx = np.array(idx)
        while len(idx) > d + 2:
            # drop the smaller end or merge smallest neighbour pair
            if abs(E[idx[0]]) < abs(E[idx[-1]]):
                idx = idx[1:]
            else:
                idx = idx[:-1]
        if len(idx) < d + 2:
            break
        emax = np.max(np.abs(E))
        emin = np.min(np.abs(E[idx]))
        u_ref = gu[idx]
        err = emax
        if emax - emin <= tol * emax:
            break
    return coef, float(err)


# ------------------------------------------------------------ the method
def exp_table(M, k, d):
    """exp(x / 2^k) on [-M, 0] as a Chebyshev series (degree d)."""
    return cheb_interp(lambda x: np.exp(x / 2.0 ** k), -M, 0.0, d)


def invpow_table(a, b, d, e=0.5, weighted=True):
    """x^(-e) on [a, b], minimising the relative error max |P(x) x^e - 1|."""
    f = lambda x: x ** (-e)
    if weighted:
        coef, err = remez(f, lambda x: x ** e, a, b, d)
    else:
        coef = cheb_interp(f, a, b, d)
        g = np.linspace(a, b, 20001)
        err = float(np.max(np.abs(cheb_eval(coef, g, a, b) * g ** e - 1)))
    return coef, err


def next_interval(n, alpha):
    """Input interval of the next normalisation (Section 5.1)."""
    return (1.0 - alpha) ** 2 / n, (1.0 + alpha) ** 2
