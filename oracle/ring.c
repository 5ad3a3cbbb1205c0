/*
 * Ring oracle: plain, single-threaded C for the integer arithmetic under
 * RNS-CKKS.  TEST INFRASTRUCTURE ONLY: this file is the slow, obviously
 * correct reference that the HIP library is checked against.  Nothing in the
 * product may include, link or call it.
 *
 * The paper treats CKKS as a black box (Section 2.2, "Functionalities";
 * Section 5.1 runs it inside an external library).  Every definition below is
 * therefore the textbook one, written out with the slowest safe arithmetic:
 * every modular product is (unsigned __int128)a*b % q.
 *
 *   negacyclic NTT   : out[i] = sum_j a_j psi^((2 brv(i)+1) j) mod q
 *                      (bit-reversed evaluation order; psi a primitive 2N-th
 *                      root of unity).  The fast loop below is the standard
 *                      Cooley-Tukey / Gentleman-Sande pair; the O(N^2)
 *                      definition is also exported so tests can pin the fast
 *                      loop to it.
 *   base conversion  : y_t = sum_i [x_i (D/d_i)^-1]_{d_i} (D/d_i) mod t
 *                      (fast, non-centred RNS base conversion).
 *   Philox4x32-10    : the counter-based generator of Salmon, Moraes, Dror
 *                      and Shaw (SC'11), used for every random draw.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <stdlib.h>

typedef uint64_t u64;
typedef uint32_t u32;
typedef unsigned __int128 u128;

static u64 mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 addmod(u64 a, u64 b, u64 q) { u128 s = (u128)a + b; return (u64)(s % q); }
static u64 submod(u64 a, u64 b, u64 q) { return a >= b ? a - b : (u64)((u128)a + q - b); }

u64 or_powmod(u64 a, u64 e, u64 q) {
    u64 r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulmod(r, a, q);
        a = mulmod(a, a, q);
        e >>= 1;
    }
    return r;
}

u64 or_invmod(u64 a, u64 q) { return or_powmod(a, q - 2, q); } /* q prime */

static u64 brv(u64 x, int bits) {
    u64 r = 0;
    for (int i = 0; i < bits; i++) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}

static int ilog2(u64 n) { int l = 0; while ((1ULL << l) < n) l++; return l; }

/* psi_brv[k] = psi^brv(k), psi_inv_brv[k] = psi^-brv(k). */
void or_psi_tables(u64 N, u64 q, u64 psi, u64* psi_brv, u64* psi_inv_brv) {
    int lg = ilog2(N);
    u64 psi_inv = or_invmod(psi, q);
    for (u64 k = 0; k < N; k++) {
        u64 e = brv(k, lg);
        psi_brv[k] = or_powmod(psi, e, q);
        psi_inv_brv[k] = or_powmod(psi_inv, e, q);
    }
}

/* Definition of the forward transform, O(N^2). */
void or_ntt_definition(const u64* a, u64* out, u64 N, u64 q, u64 psi) {
    int lg = ilog2(N);
    for (u64 i = 0; i < N; i++) {
        u64 e = 2 * brv(i, lg) + 1;
        u64 w = or_powmod(psi, e, q);
        u64 acc = 0, wp = 1;
        for (u64 j = 0; j < N; j++) {
            acc = addmod(acc, mulmod(a[j], wp, q), q);
            wp = mulmod(wp, w, q);
        }
        out[i] = acc;
    }
}

/* Cooley-Tukey, natural-order input, bit-reversed-order output. In place. */
void or_ntt_fwd(u64* a, u64 N, u64 q, const u64* psi_brv) {
    u64 t = N;
    for (u64 m = 1; m < N; m <<= 1) {
        t >>= 1;
        for (u64 i = 0; i < m; i++) {
            u64 w = psi_brv[m + i];
            u64 j1 = 2 * i * t;
            for (u64 j = j1; j < j1 + t; j++) {
                u64 u = a[j];
                u64 v = mulmod(a[j + t], w, q);
                a[j] = addmod(u, v, q);
                a[j + t] = submod(u, v, q);
            }
        }
    }
}

/* Gentleman-Sande, exact inverse of or_ntt_fwd. In place. */
void or_ntt_inv(u64* a, u64 N, u64 q, const u64* psi_inv_brv) {
    u64 t = 1;
    for (u64 m = N >> 1; m >= 1; m >>= 1) {
        for (u64 i = 0; i < m; i++) {
            u64 w = psi_inv_brv[m + i];
            u64 j1 = 2 * i * t;
            for (u64 j = j1; j < j1 + t; j++) {
                u64 u = a[j];
                u64 v = a[j + t];
                a[j] = addmod(u, v, q);
                a[j + t] = mulmod(submod(u, v, q), w, q);
            }
        }
        t <<= 1;
    }
    u64 ninv = or_invmod(N % q, q);
    for (u64 j = 0; j < N; j++) a[j] = mulmod(a[j], ninv, q);
}

/* Schoolbook product in Z_q[X]/(X^N+1). */
void or_negacyclic_mul(const u64* a, const u64* b, u64* out, u64 N, u64 q) {
    for (u64 k = 0; k < N; k++) out[k] = 0;
    for (u64 i = 0; i < N; i++)
        for (u64 j = 0; j < N; j++) {
            u64 p = mulmod(a[i], b[j], q);
            u64 k = i + j;
            if (k < N) out[k] = addmod(out[k], p, q);
            else out[k - N] = submod(out[k - N], p, q);
        }
}

/* Elementwise ops on one limb. */
void or_vec_mul(const u64* a, const u64* b, u64* out, u64 n, u64 q) {
    for (u64 i = 0; i < n; i++) out[i] = mulmod(a[i], b[i], q);
}
void or_vec_add(const u64* a, const u64* b, u64* out, u64 n, u64 q) {
    for (u64 i = 0; i < n; i++) out[i] = addmod(a[i], b[i], q);
}
void or_vec_sub(const u64* a, const u64* b, u64* out, u64 n, u64 q) {
    for (u64 i = 0; i < n; i++) out[i] = submod(a[i], b[i], q);
}
void or_vec_scalar_mul(const u64* a, u64 c, u64* out, u64 n, u64 q) {
    for (u64 i = 0; i < n; i++) out[i] = mulmod(a[i], c % q, q);
}

/*
 * Fast base conversion of coefficient-domain residues.
 *   in      : k limbs of N residues, modulo src[0..k)
 *   out     : m limbs of N residues, modulo dst[0..m)
 * y_t = sum_i [x_i * (D/d_i)^-1]_{d_i} * ((D/d_i) mod t)  mod t,  D = prod src.
 */
void or_base_convert(const u64* in, const u64* src, int k, u64* out, const u64* dst, int m, u64 N) {
    u64* inv_hat = (u64*)malloc(sizeof(u64) * k);
    u64* hat_mod = (u64*)malloc(sizeof(u64) * k * m);
    for (int i = 0; i < k; i++) {
        u64 h = 1;
        for (int j = 0; j < k; j++) if (j != i) h = mulmod(h, src[j] % src[i], src[i]);
        inv_hat[i] = or_invmod(h, src[i]);
        for (int t = 0; t < m; t++) {
            u64 g = 1;
            for (int j = 0; j < k; j++) if (j != i) g = mulmod(g, src[j] % dst[t], dst[t]);
            hat_mod[i * m + t] = g;
        }
    }
    for (int t = 0; t < m; t++) {
        u64 qt = dst[t];
        for (u64 c = 0; c < N; c++) {
            u64 acc = 0;
            for (int i = 0; i < k; i++) {
                u64 xh = mulmod(in[(u64)i * N + c], inv_hat[i], src[i]);
                acc = addmod(acc, mulmod(xh % qt, hat_mod[i * m + t], qt), qt);
            }
            out[(u64)t * N + c] = acc;
        }
    }
    free(inv_hat);
    free(hat_mod);
}

/*
 * Centred fast base conversion: as or_base_convert but each
 * [x_i (D/d_i)^-1]_{d_i} is taken in (-d_i/2, d_i/2], so the result is
 * x + u D with |u| <= k/2 and u of mean zero.  Used by ModDown, where the
 * conversion error becomes noise and must not carry a bias.
 */
void or_base_convert_centered(const u64* in, const u64* src, int k, u64* out, const u64* dst, int m, u64 N) {
    u64* inv_hat = (u64*)malloc(sizeof(u64) * k);
    u64* hat_mod = (u64*)malloc(sizeof(u64) * k * m);
    u64* D_mod = (u64*)malloc(sizeof(u64) * m);
    for (int i = 0; i < k; i++) {
        u64 h = 1;
        for (int j = 0; j < k; j++) if (j != i) h = mulmod(h, src[j] % src[i], src[i]);
        inv_hat[i] = or_invmod(h, src[i]);
        for (int t = 0; t < m; t++) {
            u64 g = 1;
            for (int j = 0; j < k; j++) if (j != i) g = mulmod(g, src[j] % dst[t], dst[t]);
            hat_mod[i * m + t] = g;
        }
    }
    for (int t = 0; t < m; t++) {
        u64 g = 1;
        for (int j = 0; j < k; j++) g = mulmod(g, src[j] % dst[t], dst[t]);
        D_mod[t] = g;
    }
    for (int t = 0; t < m; t++) {
        u64 qt = dst[t];
        for (u64 c = 0; c < N; c++) {
            u64 acc = 0;
            for (int i = 0; i < k; i++) {
                u64 xh = mulmod(in[(u64)i * N + c], inv_hat[i], src[i]);
                acc = addmod(acc, mulmod(xh % qt, hat_mod[i * m + t], qt), qt);
                if (xh > (src[i] - 1) / 2) acc = submod(acc, D_mod[t], qt);   /* xh - d_i */
            }
            out[(u64)t * N + c] = acc;
        }
    }
    free(inv_hat);
    free(hat_mod);
    free(D_mod);
}

/* Index map of X -> X^g in the NTT (bit-reversed evaluation) domain:
 * out[i] = in[perm[i]] with 2 brv(perm[i]) + 1 = (2 brv(i) + 1) g mod 2N. */
void or_automorph_perm(u64 N, u64 g, u64* perm) {
    int lg = ilog2(N);
    u64 M = 2 * N;
    for (u64 i = 0; i < N; i++) {
        u64 e = ((2 * brv(i, lg) + 1) * (g % M)) % M;
        perm[i] = brv((e - 1) / 2, lg);
    }
}

/* Philox4x32-10 (Salmon et al., SC'11): 10 rounds of the 4x32 Philox
 * S-box with multipliers 0xD2511F53, 0xCD9E8D57 and Weyl key increments
 * 0x9E3779B9, 0xBB67AE85. */
void or_philox4x32_10(const u32 ctr_in[4], const u32 key_in[2], u32 out[4]) {
    u32 c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    u32 k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        u64 p0 = (u64)0xD2511F53u * c0;
        u64 p1 = (u64)0xCD9E8D57u * c2;
        u32 hi0 = (u32)(p0 >> 32), lo0 = (u32)p0;
        u32 hi1 = (u32)(p1 >> 32), lo1 = (u32)p1;
        u32 n0 = hi1 ^ c1 ^ k0;
        u32 n1 = lo1;
        u32 n2 = hi0 ^ c3 ^ k1;
        u32 n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The draw used everywhere: key = seed, counter = (index, domain). */
static void draw(u64 seed, u64 domain, u64 index, u32 out[4]) {
    u32 key[2] = {(u32)seed, (u32)(seed >> 32)};
    u32 ctr[4] = {(u32)index, (u32)(index >> 32), (u32)domain, (u32)(domain >> 32)};
    or_philox4x32_10(ctr, key, out);
}

void or_draw_block(u64 seed, u64 domain, u64 index, u32* out4) { draw(seed, domain, index, out4); }

/* Uniform residue mod q from one 128-bit block: (w3:w2:w1:w0) mod q. */
void or_sample_uniform(u64 seed, u64 domain, u64 N, u64 q, u64* out) {
    for (u64 i = 0; i < N; i++) {
        u32 w[4];
        draw(seed, domain, i, w);
        u128 v = ((u128)w[3] << 96) | ((u128)w[2] << 64) | ((u128)w[1] << 32) | (u128)w[0];
        out[i] = (u64)(v % q);
    }
}

/* Uniform ternary: s_i from (w0 mod 3): 0 -> 0, 1 -> 1, 2 -> -1. */
void or_sample_ternary(u64 seed, u64 domain, u64 N, int64_t* out) {
    for (u64 i = 0; i < N; i++) {
        u32 w[4];
        draw(seed, domain, i, w);
        u32 r = w[0] % 3u;
        out[i] = r == 0 ? 0 : (r == 1 ? 1 : -1);
    }
}

/* Sparse ternary of Hamming weight h by a partial Fisher-Yates shuffle:
 * step t draws block t, swaps position t with t + (w1:w0 mod (N-t)), and the
 * chosen coefficient gets sign (w2 & 1 ? -1 : +1). */
void or_sample_sparse_ternary(u64 seed, u64 domain, u64 N, u64 h, int64_t* out) {
    u64* pos = (u64*)malloc(sizeof(u64) * N);
    for (u64 i = 0; i < N; i++) { pos[i] = i; out[i] = 0; }
    for (u64 t = 0; t < h; t++) {
        u32 w[4];
        draw(seed, domain, t, w);
        u64 r = ((u64)w[1] << 32) | w[0];
        u64 j = t + r % (N - t);
        u64 tmp = pos[t]; pos[t] = pos[j]; pos[j] = tmp;
        out[pos[t]] = (w[2] & 1u) ? -1 : 1;
    }
    free(pos);
}

/* Discrete Gaussian by cumulative table: u = (w1:w0); |e| = smallest k with
 * u < table[k] (table[nt-1] must be the all-ones sentinel); sign from w2&1. */
void or_sample_cdt(u64 seed, u64 domain, u64 N, const u64* table, int nt, int64_t* out) {
    for (u64 i = 0; i < N; i++) {
        u32 w[4];
        draw(seed, domain, i, w);
        u64 u = ((u64)w[1] << 32) | w[0];
        int k = 0;
        while (k < nt - 1 && u >= table[k]) k++;
        out[i] = (w[2] & 1u) ? -(int64_t)k : (int64_t)k;
    }
}
