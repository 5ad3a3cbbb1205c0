"""FP64 Softmax reference, the paper's precision metrics, and plaintext
twins of the paper's algorithms.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

* ``softmax`` is the definition (Eq. "eq:smdef"), evaluated with the shift of
  Eq. "eq:normalized_sm" so it never overflows.
* ``precision_bits`` follows Section 5.2 ("Error measurements"): the error of
  one vector is the max-norm of the difference; worst = -log2 of the largest
  error; average = -log2 of the mean error; the spread is the standard
  deviation of log2 of the per-vector errors.
* The twins run the paper's loops on plain float64 vectors, in the paper's
  order and notation:
    main_loop        -- Algorithm "alg:main_loop" / "alg:Softmax" (SM)
    softmax_b        -- Algorithm "alg:Softmax1B" (SM version B)
    aux_thread_slots -- Algorithm "alg:AuxThread" on a packed slot vector
  Each takes the exponential and the normalisation functions as arguments,
  so the same loop runs with exact functions (it must then return SM(x), the
  doubling identity Eq. "eq:doubling_sm") or with polynomial approximations.
* Packing follows Section 4: one ciphertext interleaves N0/n Softmax with
  stride N0/n; m ciphertexts hold L = m N0 / n Softmax, ciphertext j putting
  coordinate j*(n/m) + c of Softmax l in slot c*L + l.
"""
import math

import numpy as np


def softmax(x):
    """Softmax of each row of x (definition, shifted by the row maximum)."""
    x = np.asarray(x, dtype=np.float64)
    e = np.exp(x - x.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def precision_bits(y_ref, y):
    """Per-vector absolute errors and the paper's summary statistics (bits)."""
    err = np.max(np.abs(np.asarray(y_ref) - np.asarray(y)), axis=-1)
    err = np.maximum(err, 2.0 ** -60)
    return dict(
        worst=-math.log2(float(err.max())),
        mean=-math.log2(float(err.mean())),
        mean_of_bits=float(np.mean(-np.log2(err))),
        std=float(np.std(np.log2(err))),
        min_vector_bits=float(np.min(-np.log2(err))),
    )


def theorem_k(n, M):
    """k = ceil(log M - log ln n) (Theorem "th:prec_softmax")."""
    return max(1, int(math.ceil(math.log2(M) - math.log2(math.log(n)))))


def table_k(M):
    """k with range [-2^k, 0] (the practical tables of Section 3)."""
    return int(math.ceil(math.log2(M)))


def theorem_bound(n, k, p):
    """Error bound of Theorem "th:prec_softmax" and whether its premise holds."""
    eps = 2.0 ** -p
    premise = max(n * n, 2.9 * (2.08 * math.sqrt(n)) ** k) * eps <= 1.0 / 1000
    bound = 2.9 * ((2.08 * math.sqrt(n)) ** k * (n + 1) + 15.5 * n * n) * eps
    return bound, premise


# ---------------------------------------------------------------- twins
def _noise(shape, rng, eps):
    if rng is None or eps == 0.0:
        return 0.0
    return rng.uniform(-eps, eps, size=shape)


def main_loop(x, k, exp_fn=None, norm_fns=None, rng=None, eps=0.0):
    """Algorithm SM: y0 = exp(x / 2^k); k times lambda = (sum y^2)^(-1/2),
    z = lambda y, y = z^2.  Rows of x are independent Softmax inputs.

    exp_fn(t) approximates exp(t); norm_fns[j-1](s) approximates s^(-1/2).
    With rng/eps every operation other than addition gets an absolute error
    uniform in [-eps, eps] (the fixed-point model of Section 2.2)."""
    x = np.asarray(x, dtype=np.float64)
    exp_fn = exp_fn or np.exp
    y = exp_fn(x / 2.0 ** k) + _noise(x.shape, rng, eps)
    for j in range(1, k + 1):
        f = norm_fns[j - 1] if norm_fns else (lambda s: s ** -0.5)
        sq = y * y + _noise(y.shape, rng, eps)
        s = sq.sum(axis=-1, keepdims=True)
        lam = f(s) + _noise(s.shape, rng, eps)
        z = lam * y + _noise(y.shape, rng, eps)
        y = z * z + _noise(y.shape, rng, eps)
    return y


def power_loop(x, k, t, exp_fn=None, norm_fns=None):
    """Normalize-and-t-th-power (the appendix on other normalisation
    strategies): y0 = exp(x / t^k); k times lambda = (sum y^t)^(-1/t),
    y = (lambda y)^t.  With exact functions it returns SM(x), since
    SM(x) = normalize(SM(x / t)^t); norm_fns[j-1](s) approximates s^(-1/t)."""
    x = np.asarray(x, dtype=np.float64)
    exp_fn = exp_fn or np.exp
    y = exp_fn(x / float(t) ** k)
    for j in range(1, k + 1):
        f = norm_fns[j - 1] if norm_fns else (lambda s: s ** (-1.0 / t))
        s = (y ** t).sum(axis=-1, keepdims=True)
        y = (f(s) * y) ** t
    return y


def softmax_b(x, k, exp_fn=None, pow_fns=None):
    """Algorithm SM version B: Lambda = 1; y0 = exp(x/2^k); for j = 1..k:
    lambda_j = (sum y^(j-1)^2)^(-2^-j), Lambda *= lambda_j, z = Lambda y0,
    y^(j) = z^(2^j).  pow_fns[j-1](s) approximates s^(-2^-j)."""
    x = np.asarray(x, dtype=np.float64)
    exp_fn = exp_fn or np.exp
    y0 = exp_fn(x / 2.0 ** k)
    y = y0
    lam = np.ones(x.shape[:-1] + (1,))
    for j in range(1, k + 1):
        f = pow_fns[j - 1] if pow_fns else (lambda s, j=j: s ** (-(2.0 ** -j)))
        s = (y * y).sum(axis=-1, keepdims=True)
        lam = lam * f(s)
        z = lam * y0
        y = z
        for _ in range(j):
            y = y * y
    return y


# --------------------------------------------------------------- packing
def padded(n):
    """The power of two at or above n (a dimension's packing width)."""
    return 1 << (int(n) - 1).bit_length()


def pack(logits, m, slots, pad_value=None):
    """(L, n) logits -> (m, slots) slot vectors; L must equal m*slots/n2 with
    n2 = padded(n); coordinates n..n2-1 take pad_value (default: the row
    minimum's floor, i.e. any value in range; they are masked out)."""
    logits = np.asarray(logits, dtype=np.float64)
    L, n = logits.shape
    n2 = padded(n)
    if n2 > slots or m < 1 or n2 % m or L * n2 != m * slots:
        raise ValueError("bad packing shape")
    pv = float(np.min(logits)) if pad_value is None else pad_value
    per = n2 // m
    out = np.zeros((m, slots))
    for j in range(m):
        for c in range(per):
            coord = j * per + c
            out[j, c * L:(c + 1) * L] = logits[:, coord] if coord < n else pv
    return out


def unpack(slots_m, n):
    slots_m = np.asarray(slots_m)
    m, slots = slots_m.shape
    n2 = padded(n)
    L = m * slots // n2
    per = n2 // m
    out = np.zeros((L, n), dtype=slots_m.dtype)
    for j in range(m):
        for c in range(per):
            if j * per + c < n:
                out[:, j * per + c] = slots_m[j, c * L:(c + 1) * L]
    return out


def rot(v, r):
    """Left rotation of a slot vector: slot j <- slot j + r."""
    return np.roll(v, -r)


def aux_thread_slots(cts, n, inv_fn):
    """Algorithm "alg:AuxThread" over m packed slot vectors (Section 4.2):
    square and sum the m vectors, rotate-and-add with strides -L 2^t, apply
    the normalisation function, keep slots [0, L) (the mask), and broadcast
    back with strides +L 2^t.  Returns the broadcast normalisation factors."""
    cts = np.asarray(cts, dtype=np.float64)
    m, slots = cts.shape
    L = m * slots // n
    s = (cts * cts).sum(axis=0)
    t = 0
    while (L << t) < slots:
        s = s + rot(s, -(L << t))
        t += 1
    lam = inv_fn(s)
    mask = np.zeros(slots)
    mask[:L] = 1.0
    lam = lam * mask
    t = 0
    while (L << t) < slots:
        lam = lam + rot(lam, L << t)
        t += 1
    return lam


def sm_packed(cts, n, k, exp_fn=None, norm_fns=None, variant="SM"):
    """Many-ciphertext SM or SM-B on packed slot vectors (Sections 4.2, 4.3).
    The inputs are the slot vectors of x; returns the slot vectors of the
    output.  Used to pin the packing and rotation logic of the twin."""
    exp_fn = exp_fn or np.exp
    y0 = exp_fn(np.asarray(cts, dtype=np.float64) / 2.0 ** k)
    y = y0
    big = np.ones(y.shape[1])
    for j in range(1, k + 1):
        if variant == "SM":
            f = norm_fns[j - 1] if norm_fns else (lambda s: s ** -0.5)
            lam = aux_thread_slots(y, n, f)
            z = lam * y
            y = z * z
        else:
            f = norm_fns[j - 1] if norm_fns else (lambda s, j=j: s ** (-(2.0 ** -j)))
            lam = aux_thread_slots(y, n, f)
            big = big * lam
            z = big * y0
            y = z
            for _ in range(j):
                y = y * y
    return y
