"""RNS-CKKS oracle: key generation, encryption, and every homomorphic
operation the Softmax hot path uses, written plainly over numpy arrays with
the modular products done by the C core (``oracle/ring.c``).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The paper lists the functionality it needs -- KeyGen, Enc, Dec, Add, Mult,
Rot -- and the level rule of multiplication (Section 2.2, "Functionalities"
and "Levels").  It does not describe the ring arithmetic, so each operation
below follows the textbook RNS-CKKS definitions:

  * polynomials live in R_Q = Z_Q[X]/(X^N + 1), one residue row ("limb") per
    prime, in the negacyclic NTT domain (bit-reversed evaluation order);
  * level l means limbs q[0..l]; rescale divides by q[l] with centred
    rounding; the scale of a ciphertext is tracked as an FP64 number;
  * key switching is the hybrid (digit-decomposed, special-modulus) method:
    digits are consecutive blocks of `digit` primes, P = prod p[*]; ModUp
    uses the plain fast base conversion (its error is cancelled by the key),
    ModDown the centred one (its error becomes zero-mean noise);
    swk_j = (-a_j s + e_j + [t in D_j] (P mod t) s', a_j) on every prime t;
  * rotation by r applies X -> X^(5^r mod 2N) then switches from s(X^g) back
    to s; conjugation uses g = 2N - 1.

Random draws come from Philox4x32-10 with key = 64-bit seed and counter =
(index, 64-bit domain); the domain tags are documented with each sampler.
"""
import numpy as np

from . import _lib
from .encoding import encode_coeffs, decode_coeffs
from .params import find_primes, smallest_psi

# domain tags (bits 56..63 hold the purpose)
D_SECRET = 1 << 56
D_PK_A = 2 << 56
D_PK_E = 3 << 56
D_KEY_A = 4 << 56
D_KEY_E = 5 << 56
D_ENC_V = 6 << 56
D_ENC_E0 = 7 << 56
D_ENC_E1 = 8 << 56


def key_a_domain(key_id, digit, prime_index):
    return D_KEY_A | (key_id << 24) | (digit << 16) | prime_index


def key_e_domain(key_id, digit):
    return D_KEY_E | (key_id << 24) | (digit << 16)


RELIN_KEY_ID = 0


def gaussian_cdt(sigma, kmax=40):
    """table[k] = floor(2^64 * Pr(|e| <= k)) for the discrete Gaussian
    rho(x) = exp(-x^2 / (2 sigma^2)), k < kmax; last entry = 2^64 - 1."""
    import mpmath
    with mpmath.workprec(256):
        s2 = 2 * mpmath.mpf(sigma) ** 2
        rho = [mpmath.e ** (-(mpmath.mpf(k) ** 2) / s2) for k in range(200)]
        Z = rho[0] + 2 * mpmath.fsum(rho[1:])
        out = []
        acc = rho[0]
        for k in range(kmax):
            if k > 0:
                acc += 2 * rho[k]
            out.append(int(mpmath.floor(acc / Z * mpmath.mpf(2) ** 64)))
    out[-1] = (1 << 64) - 1
    return np.array([min(v, (1 << 64) - 1) for v in out], dtype=np.uint64)


class Ciphertext:
    def __init__(self, c, level, scale):
        self.c = c            # list of (level+1, N) uint64 arrays, NTT domain
        self.level = level
        self.scale = float(scale)

    def copy(self):
        return Ciphertext([x.copy() for x in self.c], self.level, self.scale)


class Context:
    """One parameter set: primes, NTT tables, keys."""

    def __init__(self, logN, q_bits, p_bits, digit, hamming, sigma=3.2, log_scale=40, **_):
        self.logN = logN
        self.N = N = 1 << logN
        self.slots = N // 2
        self.q, self.p = find_primes(logN, q_bits, p_bits)
        self.primes = self.q + self.p          # global prime index: Q then P
        self.L = len(self.q) - 1
        self.alpha = len(self.p)
        self.digit = digit
        self.dnum = (len(self.q) + digit - 1) // digit
        self.hamming = hamming
        self.sigma = sigma
        self.delta = float(2 ** log_scale)
        self.P = 1
        for pp in self.p:
            self.P *= pp
        L = _lib.lib()
        self._L = L
        self.psi = [smallest_psi(t, N) for t in self.primes]
        self.psi_brv = []
        self.psi_inv_brv = []
        for t, ps in zip(self.primes, self.psi):
            a = np.empty(N, dtype=np.uint64)
            b = np.empty(N, dtype=np.uint64)
            L.or_psi_tables(N, t, ps, a, b)
            self.psi_brv.append(a)
            self.psi_inv_brv.append(b)
        self.cdt = gaussian_cdt(sigma)
        self.keys = {}
        self.s_coeff = None

    # ------------------------------------------------------------------ ring
    def ntt(self, x, idx):
        out = np.ascontiguousarray(x, dtype=np.uint64).copy()
        self._L.or_ntt_fwd(out, self.N, self.primes[idx], self.psi_brv[idx])
        return out

    def intt(self, x, idx):
        out = np.ascontiguousarray(x, dtype=np.uint64).copy()
        self._L.or_ntt_inv(out, self.N, self.primes[idx], self.psi_inv_brv[idx])
        return out

    def mul(self, a, b, idx):
        out = np.empty(self.N, dtype=np.uint64)
        self._L.or_vec_mul(np.ascontiguousarray(a), np.ascontiguousarray(b), out, self.N, self.primes[idx])
        return out

    def add(self, a, b, idx):
        out = np.empty(self.N, dtype=np.uint64)
        self._L.or_vec_add(np.ascontiguousarray(a), np.ascontiguousarray(b), out, self.N, self.primes[idx])
        return out

    def sub(self, a, b, idx):
        out = np.empty(self.N, dtype=np.uint64)
        self._L.or_vec_sub(np.ascontiguousarray(a), np.ascontiguousarray(b), out, self.N, self.primes[idx])
        return out

    def smul(self, a, c, idx):
        out = np.empty(self.N, dtype=np.uint64)
        self._L.or_vec_scalar_mul(np.ascontiguousarray(a), int(c) % self.primes[idx], out, self.N,
                                  self.primes[idx])
        return out

    def ints_to_limb(self, coeffs, idx):
        """Signed integer coefficients -> residues mod primes[idx] (coefficient domain)."""
        t = self.primes[idx]
        return np.array([int(c) % t for c in coeffs], dtype=np.uint64)

    def small_to_ntt(self, small, idx):
        """int64 coefficients (small) -> NTT-domain limb."""
        return self.ntt(self.signed_to_limb(small, idx), idx)

    def signed_to_limb(self, v, idx):
        """int64 values with |v| < 2^62 -> residues mod primes[idx]."""
        t = np.int64(self.primes[idx])
        return (np.asarray(v, dtype=np.int64) % t).astype(np.uint64)

    def base_convert(self, limbs, src_idx, dst_idx, centered=False):
        """Fast base conversion (coefficient domain) from primes src to dst;
        centered=True takes each [x_i (D/d_i)^-1]_{d_i} in (-d_i/2, d_i/2]."""
        k = len(src_idx)
        m = len(dst_idx)
        inp = np.ascontiguousarray(np.stack(limbs).reshape(-1), dtype=np.uint64)
        src = np.array([self.primes[i] for i in src_idx], dtype=np.uint64)
        dst = np.array([self.primes[i] for i in dst_idx], dtype=np.uint64)
        out = np.empty(m * self.N, dtype=np.uint64)
        f = self._L.or_base_convert_centered if centered else self._L.or_base_convert
        f(inp, src, k, out, dst, m, self.N)
        return [out[i * self.N:(i + 1) * self.N].copy() for i in range(m)]

    def automorph_perm(self, g):
        perm = np.empty(self.N, dtype=np.uint64)
        self._L.or_automorph_perm(self.N, g, perm)
        return perm.astype(np.int64)

    # -------------------------------------------------------------- sampling
    def _sample_small(self, seed, domain, kind):
        N = self.N
        out = np.empty(N, dtype=np.int64)
        if kind == "ternary":
            self._L.or_sample_ternary(seed, domain, N, out)
        elif kind == "sparse":
            self._L.or_sample_sparse_ternary(seed, domain, N, self.hamming, out)
        elif kind == "gauss":
            self._L.or_sample_cdt(seed, domain, N, self.cdt, len(self.cdt), out)
        else:
            raise ValueError(kind)
        return out

    def _uniform(self, seed, domain, idx):
        out = np.empty(self.N, dtype=np.uint64)
        self._L.or_sample_uniform(seed, domain, self.N, self.primes[idx], out)
        return out

    # ---------------------------------------------------------------- keygen
    def keygen(self, seed, galois=()):
        """Secret, public, relinearisation and Galois keys from one seed."""
        self.seed = seed
        kind = "sparse" if self.hamming else "ternary"
        self.s_coeff = self._sample_small(seed, D_SECRET, kind)
        self.s_ntt = [self.small_to_ntt(self.s_coeff, i) for i in range(len(self.primes))]
        # public key over Q
        e = self._sample_small(seed, D_PK_E, "gauss")
        self.pk1 = [self._uniform(seed, D_PK_A | i, i) for i in range(len(self.q))]
        self.pk0 = []
        for i in range(len(self.q)):
            as_ = self.mul(self.pk1[i], self.s_ntt[i], i)
            self.pk0.append(self.add(self.sub(np.zeros(self.N, dtype=np.uint64), as_, i),
                                     self.small_to_ntt(e, i), i))
        s2 = [self.mul(self.s_ntt[i], self.s_ntt[i], i) for i in range(len(self.primes))]
        self.keys[RELIN_KEY_ID] = self.switching_key(RELIN_KEY_ID, s2)
        for g in galois:
            self.add_galois_key(g)

    def add_galois_key(self, g):
        g = int(g) % (2 * self.N)
        if g in self.keys:
            return
        perm = self.automorph_perm(g)
        sg = [self.s_ntt[i][perm] for i in range(len(self.primes))]
        self.keys[g] = self.switching_key(g, sg)

    def switching_key(self, key_id, s_target):
        """List over digits j of (b_j, a_j), each a list of limbs over Q u P."""
        key = []
        nq = len(self.q)
        for j in range(self.dnum):
            e = self._sample_small(self.seed, key_e_domain(key_id, j), "gauss")
            bj, aj = [], []
            for t in range(len(self.primes)):
                a = self._uniform(self.seed, key_a_domain(key_id, j, t), t)
                b = self.sub(self.small_to_ntt(e, t), self.mul(a, self.s_ntt[t], t), t)
                if t < nq and j * self.digit <= t < (j + 1) * self.digit:
                    pm = self.P % self.primes[t]
                    b = self.add(b, self.smul(s_target[t], pm, t), t)
                bj.append(b)
                aj.append(a)
            key.append((bj, aj))
        return key

    @staticmethod
    def galois_rot(r, N):
        return pow(5, r % (N // 2), 2 * N)

    # ------------------------------------------------------ encode / encrypt
    def encode(self, z, scale, level):
        coeffs = encode_coeffs(self.N, z, scale)
        return [self.ntt(self.ints_to_limb(coeffs, i), i) for i in range(level + 1)], coeffs

    def encrypt(self, pt_limbs, level, scale, seed):
        v = self._sample_small(seed, D_ENC_V, "ternary")
        e0 = self._sample_small(seed, D_ENC_E0, "gauss")
        e1 = self._sample_small(seed, D_ENC_E1, "gauss")
        c0, c1 = [], []
        for i in range(level + 1):
            vn = self.small_to_ntt(v, i)
            a0 = self.add(self.mul(vn, self.pk0[i], i), self.small_to_ntt(e0, i), i)
            c0.append(self.add(a0, pt_limbs[i], i))
            c1.append(self.add(self.mul(vn, self.pk1[i], i), self.small_to_ntt(e1, i), i))
        return Ciphertext([np.stack(c0), np.stack(c1)], level, scale)

    def encode_encrypt(self, z, scale, level, seed):
        pt, _ = self.encode(z, scale, level)
        return self.encrypt(pt, level, scale, seed)

    def decrypt_coeffs(self, ct):
        """Centred integer coefficients of c0 + c1 s (+ c2 s^2) mod Q_level."""
        lv = ct.level
        limbs = []
        for i in range(lv + 1):
            acc = ct.c[0][i]
            spow = self.s_ntt[i]
            for k in range(1, len(ct.c)):
                acc = self.add(acc, self.mul(ct.c[k][i], spow, i), i)
                spow = self.mul(spow, self.s_ntt[i], i)
            limbs.append(self.intt(acc, i))
        return self.crt(limbs, list(range(lv + 1)))

    def crt(self, limbs, idx):
        Q = 1
        for i in idx:
            Q *= self.primes[i]
        acc = [0] * self.N
        for limb, i in zip(limbs, idx):
            qi = self.primes[i]
            Qi = Q // qi
            c = Qi * pow(Qi % qi, -1, qi)
            lv = limb.tolist()
            for k in range(self.N):
                acc[k] += lv[k] * c
        half = Q // 2
        out = []
        for v in acc:
            v %= Q
            out.append(v - Q if v > half else v)
        return out

    def decrypt_decode(self, ct):
        return decode_coeffs(self.N, self.decrypt_coeffs(ct), ct.scale)

    # ------------------------------------------------------------ arithmetic
    def _check(self, a, b):
        if a.level != b.level:
            raise ValueError("level mismatch")

    def add_ct(self, a, b):
        self._check(a, b)
        n = max(len(a.c), len(b.c))
        out = []
        for k in range(n):
            if k < len(a.c) and k < len(b.c):
                out.append(np.stack([self.add(a.c[k][i], b.c[k][i], i) for i in range(a.level + 1)]))
            else:
                out.append((a.c[k] if k < len(a.c) else b.c[k]).copy())
        return Ciphertext(out, a.level, a.scale)

    def sub_ct(self, a, b):
        self._check(a, b)
        out = [np.stack([self.sub(a.c[k][i], b.c[k][i], i) for i in range(a.level + 1)])
               for k in range(2)]
        return Ciphertext(out, a.level, a.scale)

    def mul_plain(self, a, pt_limbs, pt_scale):
        out = [np.stack([self.mul(a.c[k][i], pt_limbs[i], i) for i in range(a.level + 1)])
               for k in range(len(a.c))]
        return Ciphertext(out, a.level, a.scale * pt_scale)

    def mul_int(self, a, c):
        """Multiply by the (signed, possibly large) integer c; scale unchanged."""
        out = [np.stack([self.smul(a.c[k][i], int(c) % self.primes[i], i) for i in range(a.level + 1)])
               for k in range(len(a.c))]
        return Ciphertext(out, a.level, a.scale)

    def add_int(self, a, c):
        """Add the constant polynomial c (an integer) to the message."""
        out = [x.copy() for x in a.c]
        for i in range(a.level + 1):
            t = self.primes[i]
            out[0][i] = self.add(out[0][i], np.full(self.N, int(c) % t, dtype=np.uint64), i)
        return Ciphertext(out, a.level, a.scale)

    def tensor(self, a, b):
        self._check(a, b)
        d0, d1, d2 = [], [], []
        for i in range(a.level + 1):
            d0.append(self.mul(a.c[0][i], b.c[0][i], i))
            d1.append(self.add(self.mul(a.c[0][i], b.c[1][i], i), self.mul(a.c[1][i], b.c[0][i], i), i))
            d2.append(self.mul(a.c[1][i], b.c[1][i], i))
        return Ciphertext([np.stack(d0), np.stack(d1), np.stack(d2)], a.level, a.scale * b.scale)

    def mod_drop(self, a, level):
        return Ciphertext([x[:level + 1].copy() for x in a.c], level, a.scale)

    def rescale(self, a):
        lv = a.level
        ql = self.q[lv]
        out = []
        for comp in a.c:
            r = self.intt(comp[lv], lv)
            half = np.uint64((ql - 1) // 2)
            # centred residue: r > (q_l - 1)/2  ->  r - q_l
            rs = np.where(r > half, r.astype(np.int64) - np.int64(ql), r.astype(np.int64))
            rows = []
            for i in range(lv):
                qi = self.q[i]
                rn = self.ntt(self.signed_to_limb(rs, i), i)
                inv = pow(ql % qi, -1, qi)
                rows.append(self.smul(self.sub(comp[i], rn, i), inv, i))
            out.append(np.stack(rows))
        return Ciphertext(out, lv - 1, a.scale / ql)

    def key_switch(self, d, level, key):
        """Hybrid key switching of the NTT-domain polynomial d (level+1 limbs).
        Returns (u0, u1) over q[0..level]."""
        return self.inner_mod_down(self.mod_up(d, level), level, key)

    def inner_mod_down(self, exts, level, key):
        """The rest of key switching after ModUp: the digits' inner product
        with the switching key over Q_level u P, then ModDown of both sums."""
        nq_l = level + 1
        p_idx = list(range(len(self.q), len(self.primes)))
        ext_idx = list(range(nq_l)) + p_idx
        acc0 = {t: np.zeros(self.N, dtype=np.uint64) for t in ext_idx}
        acc1 = {t: np.zeros(self.N, dtype=np.uint64) for t in ext_idx}
        for j, ext in enumerate(exts):
            bj, aj = key[j]
            for r, t in enumerate(ext_idx):
                acc0[t] = self.add(acc0[t], self.mul(ext[r], bj[t], t), t)
                acc1[t] = self.add(acc1[t], self.mul(ext[r], aj[t], t), t)
        return self.mod_down([acc0[t] for t in ext_idx], level), \
            self.mod_down([acc1[t] for t in ext_idx], level)

    def mod_up(self, d, level):
        """ModUp of the NTT-domain polynomial d (level+1 limbs): for each
        digit D_j (consecutive blocks of `digit` primes of q[0..level]) the
        extension of [d]_{D_j} to every prime of Q_level u P by the plain fast
        base conversion, NTT domain, rows q[0..level] then P; the digit's own
        rows are d's."""
        nq_l = level + 1
        p_idx = list(range(len(self.q), len(self.primes)))
        ext_idx = list(range(nq_l)) + p_idx
        out = []
        for j in range(self.dnum):
            dj = [t for t in range(j * self.digit, min((j + 1) * self.digit, nq_l))]
            if not dj:
                continue
            coeff = [self.intt(d[t], t) for t in dj]
            others = [t for t in ext_idx if t not in dj]
            conv = self.base_convert(coeff, dj, others)
            ext = {t: np.asarray(d[t], dtype=np.uint64).copy() for t in dj}
            for t, c in zip(others, conv):
                ext[t] = self.ntt(c, t)
            out.append(np.stack([ext[t] for t in ext_idx]))
        return out

    def mod_down(self, limbs, level):
        """(c - Conv_{P->Q}([c]_P)) * P^-1 mod q_i for limbs over q[0..level] u P."""
        nq_l = level + 1
        p_idx = list(range(len(self.q), len(self.primes)))
        cp = [self.intt(limbs[nq_l + k], t) for k, t in enumerate(p_idx)]
        conv = self.base_convert(cp, p_idx, list(range(nq_l)), centered=True)
        out = []
        for i in range(nq_l):
            cn = self.ntt(conv[i], i)
            pinv = pow(self.P % self.q[i], -1, self.q[i])
            out.append(self.smul(self.sub(limbs[i], cn, i), pinv, i))
        return np.stack(out)

    def relinearize(self, a):
        assert len(a.c) == 3
        u0, u1 = self.key_switch(a.c[2], a.level, self.keys[RELIN_KEY_ID])
        c0 = np.stack([self.add(a.c[0][i], u0[i], i) for i in range(a.level + 1)])
        c1 = np.stack([self.add(a.c[1][i], u1[i], i) for i in range(a.level + 1)])
        return Ciphertext([c0, c1], a.level, a.scale)

    def mult(self, a, b):
        """Mult of Section 2.2: tensor, relinearise, rescale (level - 1)."""
        return self.rescale(self.relinearize(self.tensor(a, b)))

    def automorph(self, a, g):
        perm = self.automorph_perm(g)
        return Ciphertext([x[:, perm].copy() for x in a.c], a.level, a.scale)

    def apply_galois(self, a, g):
        g = int(g) % (2 * self.N)
        b = self.automorph(a, g)
        u0, u1 = self.key_switch(b.c[1], a.level, self.keys[g])
        c0 = np.stack([self.add(b.c[0][i], u0[i], i) for i in range(a.level + 1)])
        return Ciphertext([c0, u1], a.level, a.scale)

    def rotate(self, a, r):
        """Left rotation of the slots by r (slot j <- slot j + r)."""
        return self.apply_galois(a, self.galois_rot(r, self.N))

    def conjugate(self, a):
        return self.apply_galois(a, 2 * self.N - 1)

    def rotate_hoisted(self, a, rots):
        """Rotations of one ciphertext by several offsets with one ModUp
        (hoisting, Halevi-Shoup): the ModUp digits of c1 are formed once; for
        each offset the automorphism, an NTT-domain permutation of the
        coefficients' evaluations, is applied to every extended row of every
        digit and to c0, followed by the inner product with that offset's key
        and ModDown.  The approximate base conversion does not commute
        exactly with the automorphism (a negated coefficient converts to a
        different multiple of the digit's modulus), so the words differ from
        rotate()'s while the values agree."""
        level = a.level
        exts = self.mod_up(a.c[1], level)
        out = []
        for r in rots:
            g = self.galois_rot(r, self.N)
            perm = self.automorph_perm(g)
            u0, u1 = self.inner_mod_down([e[:, perm] for e in exts], level, self.keys[g])
            c0 = np.stack([self.add(a.c[0][i][perm], u0[i], i) for i in range(level + 1)])
            out.append(Ciphertext([c0, u1], level, a.scale))
        return out

    def mod_raise(self, a, level):
        """Lift a level-0 ciphertext to q[0..level] with the centred residue."""
        assert a.level == 0
        q0 = self.q[0]
        out = []
        for comp in a.c:
            x = self.intt(comp[0], 0)
            xs = np.where(x > np.uint64((q0 - 1) // 2), x.astype(np.int64) - np.int64(q0),
                          x.astype(np.int64))
            rows = [comp[0].copy()]
            for i in range(1, level + 1):
                rows.append(self.ntt(self.signed_to_limb(xs, i), i))
            out.append(np.stack(rows))
        return Ciphertext(out, level, a.scale)

    def monomial_ntt(self, k, idx):
        """NTT of X^k (k in [0, 2N))."""
        coeff = np.zeros(self.N, dtype=np.uint64)
        k %= 2 * self.N
        if k < self.N:
            coeff[k] = 1
        else:
            coeff[k - self.N] = self.primes[idx] - 1
        return self.ntt(coeff, idx)

    def mul_monomial(self, a, k):
        out = []
        for comp in a.c:
            out.append(np.stack([self.mul(comp[i], self.monomial_ntt(k, i), i) for i in range(a.level + 1)]))
        return Ciphertext(out, a.level, a.scale)
