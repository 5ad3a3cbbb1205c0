"""Oracle parameter derivation: NTT-friendly primes and canonical roots.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper runs CKKS through an external library (Section 5.1) and prints only
the totals of its parameter set (Table "tab:fgb_data": N = 2^16, log QP =
1555, Hamming weight 192).  The choices here are ours and are stated once:

* prime rule: for a bit size b, candidates are 2^b + 1 + j*2N for
  j = 1, -1, 2, -2, ...; the chain takes, in order q[0..L] then p[0..a-1], the
  next candidate of its size that is prime and not yet used;
* psi: the smallest primitive 2N-th root of unity modulo q (as an integer),
  i.e. the minimum over g^(2i+1), i < N, for any primitive root g.
"""
import sympy


def find_primes(logN, q_bits, p_bits):
    N = 1 << logN
    step = 2 * N
    used = set()
    cursor = {}

    def next_prime(b):
        j = cursor.get(b, 0)
        while True:
            # order j -> +1, -1, +2, -2, ...
            k = j // 2 + 1
            sign = 1 if j % 2 == 0 else -1
            j += 1
            cand = (1 << b) + 1 + sign * k * step
            if cand in used or cand < 3:
                continue
            if sympy.isprime(cand):
                cursor[b] = j
                used.add(cand)
                return cand

    q = [next_prime(b) for b in q_bits]
    p = [next_prime(b) for b in p_bits]
    return q, p


def smallest_psi(q, N):
    """Smallest x in [2, q) with x of multiplicative order exactly 2N."""
    M = 2 * N
    assert (q - 1) % M == 0
    # a generator of the order-2N subgroup: x^((q-1)/2N) for the first x
    # whose image has order 2N (order 2N <=> image^N == -1)
    x = 2
    while True:
        g = pow(x, (q - 1) // M, q)
        if pow(g, N, q) == q - 1:
            break
        x += 1
    best = g
    g2 = g * g % q
    cur = g
    for _ in range(N):
        if cur < best:
            best = cur
        cur = cur * g2 % q
    return best
