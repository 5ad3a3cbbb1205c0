// Homomorphic operations on batches of ciphertexts (Section 2.2,
// "Functionalities" and "Levels": Add, Mult with level min(l1, l2) - 1, Rot).
// Every operation runs over all m ciphertexts of a batch in one launch per
// kernel; a batch with m = 1 may be broadcast against a larger one.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "host.h"

namespace hs {

static void check_scales(double a, double b, const char* op) {
    if (!(std::fabs(a / b - 1.0) < 1e-9)) {
        char msg[160];
        std::snprintf(msg, sizeof msg, "%s: operands have different scales (2^%.9f vs 2^%.9f)", op, std::log2(a),
                      std::log2(b));
        throw Error(E_SCALE, msg);
    }
}

static Rows comp_rows_bcast(const Context& c, const Ct& a, int comp, int m_target) {
    Rows r = c.comp_rows(a, comp);
    if (a.m == 1 && m_target > 1) {
        r.gstride = 0;
        r.ngroups = m_target;
    }
    return r;
}

void op_add_inplace(Context& c, Ct& a, const Ct& b) {
    HS_REQUIRE(a.level == b.level, E_LEVEL, "add: levels differ");
    HS_REQUIRE(b.m == a.m || b.m == 1, E_ARG, "add: batch sizes differ");
    HS_REQUIRE(b.ncomp <= a.ncomp, E_ARG, "add: component count");
    check_scales(a.scale, b.scale, "add");
    c.count(OC_ADD, a.level, a.m * b.ncomp / 2.0);
    for (int k = 0; k < b.ncomp; k++) {
        Rows o = c.comp_rows(a, k);
        k_add(c.T, o, o, comp_rows_bcast(c, b, k, a.m), c.stream);
    }
}

void op_sub_inplace(Context& c, Ct& a, const Ct& b) {
    HS_REQUIRE(a.level == b.level, E_LEVEL, "sub: levels differ");
    HS_REQUIRE(b.m == a.m || b.m == 1, E_ARG, "sub: batch sizes differ");
    HS_REQUIRE(b.ncomp <= a.ncomp, E_ARG, "sub: component count");
    check_scales(a.scale, b.scale, "sub");
    c.count(OC_ADD, a.level, a.m * b.ncomp / 2.0);
    for (int k = 0; k < b.ncomp; k++) {
        Rows o = c.comp_rows(a, k);
        k_sub(c.T, o, o, comp_rows_bcast(c, b, k, a.m), c.stream);
    }
}

Ct op_add(Context& c, const Ct& a, const Ct& b) {
    Ct o = ct_copy(c, a);
    op_add_inplace(c, o, b);
    return o;
}

Ct op_sub(Context& c, const Ct& a, const Ct& b) {
    Ct o = ct_copy(c, a);
    op_sub_inplace(c, o, b);
    return o;
}

void op_neg_inplace(Context& c, Ct& a) {
    Rows r = c.ct_rows(a);
    k_neg(c.T, r, r, c.stream);
}

void op_mul_residues_inplace(Context& c, Ct& a, const std::vector<u64>& res) {
    c.count(OC_PTMUL, a.level, a.m * a.ncomp / 2.0);
    RowConsts rc = c.shoup_consts(std::vector<u64>(res.begin(), res.begin() + a.level + 1), 0);
    Rows r = c.ct_rows(a);
    k_mul_row_const(c.T, r, r, rc, c.stream);
}

static std::vector<u64> int_residues(const Context& c, long long k, int level) {
    std::vector<u64> r(level + 1);
    for (int i = 0; i <= level; i++) {
        const u64 q = c.primes[i];
        const u64 m = (u64)(k < 0 ? -(k + 1) : k) % q;  // |k| - 1 for negatives avoids overflow
        if (k >= 0) r[i] = m;
        else r[i] = (q - (m + 1) % q) % q;
    }
    return r;
}

void op_mul_int_inplace(Context& c, Ct& a, long long k) { op_mul_residues_inplace(c, a, int_residues(c, k, a.level)); }

// residues of the integer value of the (integral) double v
static std::vector<u64> double_residues(const Context& c, double v, int level) {
    std::vector<u64> r(level + 1);
    const bool neg = v < 0;
    const double a = std::fabs(v);
    int e = 0;
    double mant = 0;
    u64 mi = 0;
    bool small = a < 9.2e18;
    if (!small) {
        mant = std::frexp(a, &e);
        mi = (u64)std::ldexp(mant, 53);
        e -= 53;
    }
    for (int i = 0; i <= level; i++) {
        const u64 q = c.primes[i];
        u64 mag = small ? (u64)a % q : mulmod_h(mi % q, powmod_h(2, (u64)e, q), q);
        r[i] = (neg && mag) ? q - mag : mag;
    }
    return r;
}

void op_add_const_inplace(Context& c, Ct& a, double v) {
    const double K = std::rint(v * a.scale);
    std::vector<u64> res = double_residues(c, K, a.level);
    RowConsts rc = c.shoup_consts(res, 0);
    Rows r = c.comp_rows(a, 0);
    k_add_row_const(c.T, r, r, rc, c.stream);
}

// Rescale of a into out (a.m a.ncomp groups of l rows, l = a.level): the
// rows are written, nothing else; returns the output scale.
static double rescale_into(Context& c, const Ct& a, u64* out) {
    HS_REQUIRE(a.level >= 1, E_LEVEL, "rescale: no level left");
    const int l = a.level;
    const int np_ = a.m * a.ncomp;
    const size_t N = c.N;
    u64* last = c.alloc_words((size_t)np_ * N);
    u64* lifted = c.alloc_words((size_t)np_ * l * N);
    Rows in_last{a.d + (size_t)l * N, np_, 1, (size_t)(l + 1) * N, 1, l, c.nq};
    Rows r_last{last, np_, 1, N, 1, l, c.nq};
    k_ntt_from(c.T, r_last, in_last, true, c.stream);
    Rows r_lift{lifted, np_, l, (size_t)l * N, l, 0, c.nq};
    c.count(OC_RESCALE, l, np_ / 2.0);
    std::vector<u64> inv(l);
    for (int i = 0; i < l; i++) inv[i] = invmod_h(c.primes[l] % c.primes[i], c.primes[i]);
    // out = (a - NTT(lifted)) q_l^-1, fused into the transform's last pass
    NttEpilogue e;
    e.c = c.shoup_consts(inv, 0);
    e.out[0] = out;
    e.out_gs[0] = (size_t)l * N;
    e.a = a.d;
    e.a_gs = (size_t)(l + 1) * N;
    // the transform reads the dropped row, lifted (centred) to each prime
    NttLift lf;
    lf.base = last;
    lf.gs = N;
    lf.src_prime = l;
    k_ntt_epilogue(c.T, r_lift, e, c.stream, &lf);
    c.free_words(last);
    c.free_words(lifted);
    return a.scale / (double)c.primes[l];
}

Ct op_rescale(Context& c, const Ct& a) {
    HS_REQUIRE(a.level >= 1, E_LEVEL, "rescale: no level left");
    Ct o = ct_alloc(c, a.m, a.ncomp, a.level - 1);
    o.scale = rescale_into(c, a, o.d);
    return o;
}

Ct op_mul_const(Context& c, const Ct& a, double v, double target_scale) {
    const double S = target_scale * (double)c.primes[a.level] / a.scale;
    const double K = std::rint(v * S);
    Ct t = ct_copy(c, a);
    op_mul_residues_inplace(c, t, double_residues(c, K, a.level));
    Ct o = op_rescale(c, t);
    ct_free(c, t);
    o.scale = target_scale;
    return o;
}

Ct op_mul_plain(Context& c, const Ct& a, const u64* pt, double pt_scale, bool rescale) {
    c.count(OC_PTMUL, a.level, a.m * a.ncomp / 2.0);
    Ct o = ct_alloc(c, a.m, a.ncomp, a.level);
    Rows rp{const_cast<u64*>(pt), a.m * a.ncomp, a.level + 1, 0, a.level + 1, 0, c.nq};
    k_mul(c.T, c.ct_rows(o), c.ct_rows(a), rp, c.stream);
    o.scale = a.scale * pt_scale;
    if (!rescale) return o;
    Ct r = op_rescale(c, o);
    ct_free(c, o);
    return r;
}

Ct op_tensor(Context& c, const Ct& a, const Ct& b) {
    HS_REQUIRE(a.ncomp == 2 && b.ncomp == 2, E_ARG, "tensor: degree-1 inputs expected");
    HS_REQUIRE(a.level == b.level, E_LEVEL, "tensor: levels differ");
    HS_REQUIRE(b.m == a.m || b.m == 1, E_ARG, "tensor: batch sizes differ");
    c.count(OC_TENSOR, a.level, a.m);
    Ct d = ct_alloc(c, a.m, 3, a.level);
    d.scale = a.scale * b.scale;
    const size_t cw = a.comp_words(c.N);
    Rows rd{d.d, a.m, a.level + 1, d.ct_words(c.N), a.level + 1, 0, c.nq};
    Rows ra{a.d, a.m, a.level + 1, a.ct_words(c.N), a.level + 1, 0, c.nq};
    Rows rb{b.d, a.m, a.level + 1, b.m == 1 ? 0 : b.ct_words(c.N), a.level + 1, 0, c.nq};
    k_tensor(c.T, rd, ra, rb, cw, cw, cw, c.stream);
    return d;
}

Ct op_square_sum(Context& c, const Ct& a) {
    HS_REQUIRE(a.ncomp == 2, E_ARG, "square_sum: degree-1 inputs expected");
    c.count(OC_TENSOR, a.level, a.m);
    c.count(OC_ADD, a.level, 1.5 * (a.m - 1));
    Ct d = ct_alloc(c, 1, 3, a.level);
    d.scale = a.scale * a.scale;
    Rows ra{a.d, a.m, a.level + 1, a.ct_words(c.N), a.level + 1, 0, c.nq};
    k_square_sum(c.T, d.d, d.comp_words(c.N), ra, a.comp_words(c.N), c.stream);
    return d;
}

// J sums: output j = sum over ciphertexts [j m, (j + 1) m) of a of their
// squares (degree 2), m = a.m / J
Ct op_square_sum_jobs(Context& c, const Ct& a, int jobs) {
    HS_REQUIRE(a.ncomp == 2, E_ARG, "square_sum: degree-1 inputs expected");
    HS_REQUIRE(jobs >= 1 && a.m % jobs == 0, E_ARG, "square_sum: batch not divisible into jobs");
    const int m = a.m / jobs;
    c.count(OC_TENSOR, a.level, a.m);
    c.count(OC_ADD, a.level, 1.5 * (a.m - jobs));
    Ct d = ct_alloc(c, jobs, 3, a.level);
    d.scale = a.scale * a.scale;
    for (int j = 0; j < jobs; j++) {
        Rows ra{a.d + (size_t)j * m * a.ct_words(c.N), m, a.level + 1, a.ct_words(c.N), a.level + 1, 0, c.nq};
        k_square_sum(c.T, d.d + (size_t)j * d.ct_words(c.N), d.comp_words(c.N), ra, a.comp_words(c.N), c.stream);
    }
    return d;
}

// Hybrid key switching of the m polynomials d (level l, NTT domain):
// ModUp per digit, inner product with the key, ModDown.  Writes
// out_k[g] = (add_k[g] +) ModDown(acc_k[g]) for k = 0, 1.
// ModUp of d (NTT domain, m groups of level+1 rows): digit j of every group
// lifted to Q_level u P by fast base conversion and returned in the NTT
// domain, [m][beta][E][N] with E = level + 1 + n_p.
static u64* ks_modup(Context& c, const Rows& d, int level) {
    const int m = d.ngroups;
    const int l = level;
    const int nql = l + 1;
    const int E = nql + c.np;
    const int beta = (nql + c.prm.digit - 1) / c.prm.digit;
    const size_t N = c.N;
    // the extension first, then the coefficient-domain copy of d (freed
    // first, so its block rejoins the free space behind the extension)
    u64* ext = c.alloc_words((size_t)m * beta * E * N);
    u64* dc = c.alloc_words((size_t)m * nql * N);
    Rows rdc{dc, m, nql, (size_t)nql * N, nql, 0, c.nq};
    k_ntt_from(c.T, rdc, d, true, c.stream);
    const size_t xg = (size_t)beta * E * N;
    // at N = 2^16 the digit's own rows are taken from d (already in the NTT
    // domain) and the one forward launch skips them; elsewhere they are
    // copied in the coefficient domain and transformed with the others
    const bool skip = c.logN == 16;
    for (int j = 0; j < beta; j++) {
        // every row of digit j's extension: the conversion writes the other
        // primes and copies the digit's own rows
        u64* xj = ext + (size_t)j * E * N;
        const ConvDev& cv = c.modup_tables(l, j);
        k_base_convert(c.T, cv.t, xj, xg, dc, (size_t)nql * N, m, c.stream, skip ? d.base : nullptr, d.gstride);
    }
    c.free_words(dc);
    // one launch for every row of every digit (a launch per row range would
    // under-fill the GPU for single ciphertexts)
    NttSkip sk;
    if (skip) {
        sk.per = beta;
        sk.digit = c.prm.digit;
        sk.nql = nql;
    }
    k_ntt_skip(c.T, Rows{ext, m * beta, E, (size_t)E * N, nql, 0, c.nq}, sk, c.stream);
    return ext;
}

// Inner product of the lifted digits with the key, then ModDown (centred
// conversion of the P part, times P^-1); out_k = (add_k +) result_k.
static void ks_finish(Context& c, const u64* ext, int m, int level, const KeyList& keys, u64* out0, u64* out1,
                      size_t out_gstride, const Rows* add0, const Rows* add1) {
    const int l = level;
    const int nql = l + 1;
    const int E = nql + c.np;
    const int beta = (nql + c.prm.digit - 1) / c.prm.digit;
    const size_t N = c.N;
    c.count(OC_KS, l, m);
    // inner product with the key: acc [m][2][E][N]
    u64* acc = c.alloc_words((size_t)m * 2 * E * N);
    HS_REQUIRE(keys.n * keys.per == m, E_ARG, "key switch: key list does not cover the batch");
    k_key_inner(c.T, acc, ext, keys, beta, E, nql, c.nq + c.np, c.nq, c.stream);
    // ModDown
    Rows accp{acc + (size_t)nql * N, 2 * m, c.np, (size_t)E * N, 0, 0, c.nq};
    k_ntt(c.T, accp, true, c.stream);
    u64* conv = c.alloc_words((size_t)2 * m * nql * N);
    const ConvDev& md = c.moddown_tables(l);
    k_base_convert(c.T, md.t, conv, (size_t)nql * N, acc, (size_t)E * N, 2 * m, c.stream);
    Rows rconv{conv, 2 * m, nql, (size_t)nql * N, nql, 0, c.nq};
    // out_k = (add_k +) (acc_k - NTT(conv_k)) P^-1, fused into the transform's
    // last pass; both acc's Q rows (through the key) and the conversion's
    // outputs (through its constants) already carry the factor P^-1.  Group G
    // of conv is component G mod 2 of ciphertext G / 2
    NttEpilogue e;
    e.mul = false;
    e.split = 2;
    e.a = acc;
    e.a_gs = (size_t)E * N;
    for (int k = 0; k < 2; k++) {
        e.out[k] = k == 0 ? out0 : out1;
        e.out_gs[k] = out_gstride;
        const Rows* add = k == 0 ? add0 : add1;
        if (add) {
            HS_REQUIRE(add->ngroups == m && add->rpg == nql, E_ARG, "key switch: addend shape");
            e.d[k] = add->base;
            e.d_gs[k] = add->gstride;
        }
    }
    k_ntt_epilogue(c.T, rconv, e, c.stream);
    c.free_words(acc);
    c.free_words(conv);
}

u64* op_modup_rows(Context& c, const Rows& d, int level) { return ks_modup(c, d, level); }

// ModDown of one polynomial over Q_l u P (NTT domain, rows q_0..q_l then
// p_0..p_{alpha-1}): the Q rows are first multiplied by P^-1 (the form the
// key inner product leaves them in, its keys carrying that factor), then the
// same conversion and fused epilogue as the key switch.
void op_mod_down_rows(Context& c, const u64* in, int level, u64* out) {
    const int nql = level + 1;
    const int E = nql + c.np;
    const size_t N = c.N;
    u64* acc = c.alloc_words((size_t)E * N);
    Rows src{const_cast<u64*>(in), 1, E, (size_t)E * N, nql, 0, c.nq};
    Rows racc{acc, 1, E, (size_t)E * N, nql, 0, c.nq};
    k_copy_rows(c.T, racc, src, c.stream);
    std::vector<u64> pinv(nql);
    for (int i = 0; i < nql; i++) pinv[i] = invmod_h(c.P_mod[i], c.primes[i]);
    Rows accq{acc, 1, nql, (size_t)E * N, nql, 0, c.nq};
    k_mul_row_const(c.T, accq, accq, c.shoup_consts(pinv, 0), c.stream);
    Rows accp{acc + (size_t)nql * N, 1, c.np, (size_t)E * N, 0, 0, c.nq};
    k_ntt(c.T, accp, true, c.stream);
    u64* conv = c.alloc_words((size_t)nql * N);
    const ConvDev& md = c.moddown_tables(level);
    k_base_convert(c.T, md.t, conv, (size_t)nql * N, acc, (size_t)E * N, 1, c.stream);
    Rows rconv{conv, 1, nql, (size_t)nql * N, nql, 0, c.nq};
    NttEpilogue e;
    e.mul = false;
    e.split = 1;
    e.a = acc;
    e.a_gs = (size_t)E * N;
    e.out[0] = out;
    e.out_gs[0] = (size_t)nql * N;
    k_ntt_epilogue(c.T, rconv, e, c.stream);
    c.free_words(acc);
    c.free_words(conv);
}

void key_switch(Context& c, const Rows& d, int level, const u64* key, u64* out0, u64* out1, size_t out_gstride,
                const Rows* add0, const Rows* add1) {
    u64* ext = ks_modup(c, d, level);
    KeyList kl;
    kl.key[0] = key;
    kl.n = 1;
    kl.per = d.ngroups;
    ks_finish(c, ext, d.ngroups, level, kl, out0, out1, out_gstride, add0, add1);
    c.free_words(ext);
}

// relinearisation of d into o (allocated by the caller, d's shape with two
// components)
static void relin_into(Context& c, const Ct& d, Ct& o) {
    HS_REQUIRE(d.ncomp == 3, E_ARG, "relin: degree-2 input expected");
    HS_REQUIRE(has_key(c, 0), E_KEY, "relinearisation key missing");
    o.scale = d.scale;
    Rows d2 = c.comp_rows(d, 2);
    Rows a0 = c.comp_rows(d, 0), a1 = c.comp_rows(d, 1);
    key_switch(c, d2, d.level, c.keys.at(0), o.d, o.d + o.comp_words(c.N), o.ct_words(c.N), &a0, &a1);
}

Ct op_relin(Context& c, const Ct& d) {
    HS_REQUIRE(d.ncomp == 3, E_ARG, "relin: degree-2 input expected");
    HS_REQUIRE(has_key(c, 0), E_KEY, "relinearisation key missing");
    Ct o = ct_alloc(c, d.m, 2, d.level);
    relin_into(c, d, o);
    return o;
}

// Mult (tensor, relinearisation and, when rescale is set, rescale) of two
// degree-1 ciphertexts of one level, written to out (two components at the
// output level); intermediates come from the current arena.  The kernels and
// their order are op_mult's (and hs_mult_relin's without rescale), so the
// words are the same.  Returns the output scale.
double op_mult_into(Context& c, const Ct& a, const Ct& b, bool rescale, u64* out) {
    HS_REQUIRE(a.level == b.level, E_LEVEL, "mult: levels differ");
    Ct d = op_tensor(c, a, b);
    Ct r;
    r.m = d.m;
    r.ncomp = 2;
    r.level = d.level;
    r.d = rescale ? c.alloc_words(r.ct_words(c.N)) : out;
    relin_into(c, d, r);
    ct_free(c, d);
    if (!rescale) return r.scale;
    const double s = rescale_into(c, r, out);
    c.free_words(r.d);
    return s;
}

Ct op_mult(Context& c, const Ct& a, const Ct& b) {
    const Ct* pa = &a;
    const Ct* pb = &b;
    Ct ta, tb;
    if (a.level > b.level) {
        ta = ct_drop(c, a, b.level);
        pa = &ta;
    } else if (b.level > a.level) {
        tb = ct_drop(c, b, a.level);
        pb = &tb;
    }
    Ct d = op_tensor(c, *pa, *pb);
    if (ta.d) ct_free(c, ta);
    if (tb.d) ct_free(c, tb);
    Ct r = op_relin(c, d);
    ct_free(c, d);
    Ct o = op_rescale(c, r);
    ct_free(c, r);
    return o;
}

Ct op_apply_galois(Context& c, const Ct& a, int g) {
    HS_REQUIRE(a.ncomp == 2, E_ARG, "automorphism: degree-1 input expected");
    g = ((g % (2 * c.N)) + 2 * c.N) % (2 * c.N);
    HS_REQUIRE(has_key(c, g), E_KEY, "Galois key missing");
    Ct b = ct_alloc(c, a.m, 2, a.level);
    k_permute(c.T, c.ct_rows(b), c.ct_rows(a), c.perm(g), c.stream);
    Ct o = ct_alloc(c, a.m, 2, a.level);
    o.scale = a.scale;
    Rows b0 = c.comp_rows(b, 0);
    Rows b1 = c.comp_rows(b, 1);
    key_switch(c, b1, a.level, c.keys.at(g), o.d, o.d + o.comp_words(c.N), o.ct_words(c.N), &b0, nullptr);
    ct_free(c, b);
    return o;
}

Ct op_rotate(Context& c, const Ct& a, int r) {
    if (((r % (c.N / 2)) + c.N / 2) % (c.N / 2) == 0) return ct_copy(c, a);
    return op_apply_galois(c, a, galois_rot(r, c.N));
}

Ct op_conjugate(Context& c, const Ct& a) { return op_apply_galois(c, a, 2 * c.N - 1); }

// Rotations of one ciphertext batch sharing a single ModUp (hoisting): the
// automorphism is a slot permutation in the NTT domain, the same for every
// prime, so it commutes with the lifted digits, which are a valid lift of the
// rotated digits.  The results decrypt like op_rotate's; their words differ
// (another valid lift), so this is used where only the values matter.  All R
// rotations go through one permutation launch, one inner product (a key per
// rotation) and one ModDown; the result holds R a.m ciphertexts,
// rotation-major.  No r may be a multiple of the slot count.
Ct op_rotate_hoisted_batch(Context& c, const Ct& a, const std::vector<int>& rots) {
    HS_REQUIRE(a.ncomp == 2, E_ARG, "automorphism: degree-1 input expected");
    const int R = (int)rots.size();
    HS_REQUIRE(R >= 1 && R <= kMaxKeys, E_ARG, "hoisted rotations: 1 to 32 per batch");
    const int half = c.N / 2;
    const int nql = a.level + 1;
    const int E = nql + c.np;
    const int beta = (nql + c.prm.digit - 1) / c.prm.digit;
    const size_t N = c.N;
    KeyList kl;
    PermList pl;
    kl.n = pl.n = R;
    for (int i = 0; i < R; i++) {
        HS_REQUIRE(((rots[i] % half) + half) % half != 0, E_ARG, "hoisted rotations: zero rotation");
        const int g = galois_rot(rots[i], c.N);
        HS_REQUIRE(has_key(c, g), E_KEY, "Galois key missing");
        kl.key[i] = c.keys.at(g);
        pl.perm[i] = c.perm(g);
    }
    u64* ext = ks_modup(c, c.comp_rows(a, 1), a.level);            // [m][beta][E][N]
    u64* extg = c.alloc_words((size_t)R * a.m * beta * E * N);      // [R][m][beta][E][N]
    pl.per = a.m * beta;
    k_permute_multi(c.T, Rows{extg, R * a.m * beta, E, (size_t)E * N, E, 0, c.nq},
                    Rows{ext, a.m * beta, E, (size_t)E * N, E, 0, c.nq}, pl, c.stream);
    c.free_words(ext);
    Ct b0 = ct_alloc(c, R * a.m, 1, a.level);                       // rotated first components
    pl.per = a.m;
    k_permute_multi(c.T, c.ct_rows(b0), c.comp_rows(a, 0), pl, c.stream);
    Ct o = ct_alloc(c, R * a.m, 2, a.level);
    o.scale = a.scale;
    kl.per = a.m;
    Rows rb0 = c.comp_rows(b0, 0);
    ks_finish(c, extg, R * a.m, a.level, kl, o.d, o.d + o.comp_words(N), o.ct_words(N), &rb0, nullptr);
    ct_free(c, b0);
    c.free_words(extg);
    return o;
}

// Automorphisms of a batch: block i (per ciphertexts) by Galois element
// gal[i], each exactly as op_apply_galois, with one permutation, ModUp,
// inner product and ModDown for the whole batch.
Ct op_galois_batch(Context& c, const Ct& a, const std::vector<int>& gal, int per) {
    HS_REQUIRE(a.ncomp == 2, E_ARG, "automorphism: degree-1 input expected");
    const int G = (int)gal.size();
    HS_REQUIRE(G >= 1 && G <= kMaxKeys && per >= 1 && a.m == G * per, E_ARG, "automorphism batch: bad shape");
    KeyList kl;
    PermList pl;
    kl.n = pl.n = G;
    kl.per = pl.per = per;
    for (int i = 0; i < G; i++) {
        const int g = ((gal[i] % (2 * c.N)) + 2 * c.N) % (2 * c.N);
        HS_REQUIRE(has_key(c, g), E_KEY, "Galois key missing");
        kl.key[i] = c.keys.at(g);
        pl.perm[i] = c.perm(g);
    }
    const size_t N = c.N;
    Ct b = ct_alloc(c, a.m, 2, a.level);
    for (int k = 0; k < 2; k++) k_permute_multi(c.T, c.comp_rows(b, k), c.comp_rows(a, k), pl, c.stream);
    u64* ext = ks_modup(c, c.comp_rows(b, 1), a.level);
    Ct o = ct_alloc(c, a.m, 2, a.level);
    o.scale = a.scale;
    Rows b0 = c.comp_rows(b, 0);
    ks_finish(c, ext, a.m, a.level, kl, o.d, o.d + o.comp_words(N), o.ct_words(N), &b0, nullptr);
    c.free_words(ext);
    ct_free(c, b);
    return o;
}

Ct op_mod_raise(Context& c, const Ct& a, int level) {
    HS_REQUIRE(a.level == 0, E_LEVEL, "ModRaise expects a level-0 ciphertext");
    HS_REQUIRE(level >= 1 && level <= c.L, E_LEVEL, "ModRaise target level");
    const size_t N = c.N;
    const int np_ = a.m * a.ncomp;
    Ct o = ct_alloc(c, a.m, a.ncomp, level);
    o.scale = a.scale;
    Rows r0{o.d, np_, 1, (size_t)(level + 1) * N, 1, 0, c.nq};
    k_copy_rows(c.T, r0, c.ct_rows(a), c.stream);
    u64* coef = c.alloc_words((size_t)np_ * N);
    Rows rc{coef, np_, 1, N, 1, 0, c.nq};
    k_ntt_from(c.T, rc, c.ct_rows(a), true, c.stream);
    Rows up{o.d + N, np_, level, (size_t)(level + 1) * N, level, 1, c.nq};
    k_lift_centered(c.T, up, coef, N, 0, c.stream);
    k_ntt(c.T, up, false, c.stream);
    c.free_words(coef);
    return o;
}

Ct op_mul_monomial(Context& c, const Ct& a, int k) {
    k = ((k % (2 * c.N)) + 2 * c.N) % (2 * c.N);
    auto& cache = c.monomials;
    const int key = k;
    u64* mono;
    auto it = cache.find(key);
    if (it == cache.end()) {
        const size_t w = (size_t)(c.L + 1) * c.N;
        std::vector<u64> h(w, 0);
        for (int i = 0; i <= c.L; i++) {
            if (k < c.N) h[(size_t)i * c.N + k] = 1;
            else h[(size_t)i * c.N + (k - c.N)] = c.primes[i] - 1;
        }
        mono = (u64*)c.persistent_alloc(w * 8, "monomial");
        c.upload(mono, h.data(), w * 8);
        k_ntt(c.T, c.rows(mono, 1, c.L + 1, w), false, c.stream);
        cache[key] = mono;
    } else {
        mono = it->second;
    }
    c.count(OC_PTMUL, a.level, a.m * a.ncomp / 2.0);
    Ct o = ct_alloc(c, a.m, a.ncomp, a.level);
    o.scale = a.scale;
    Rows rp{mono, a.m * a.ncomp, a.level + 1, 0, a.level + 1, 0, c.nq};
    k_mul(c.T, c.ct_rows(o), c.ct_rows(a), rp, c.stream);
    return o;
}

}  // namespace hs
