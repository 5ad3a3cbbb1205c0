// CKKS bootstrapping, coefficient-to-slot first (Section 2.2, "Levels": a
// ciphertext at its bottom level is refreshed to a full budget).  The paper
// uses an external library's bootstrapping and gives only its cost and
// precision (Section 5.1, Table "tab:fgb_data"); this pipeline is the
// standard one for full-slot CKKS and is this library's own design:
//
//  1. scale the message so that |m| ~ q0 / 2^9 at the stated bound, keep
//     the q0 limb and lift it to every Q prime (ModRaise): the result
//     decrypts to t = m + q0 I with |I| <= K;
//  2. CoeffToSlot: the inverse special FFT (without its bit reversal) as a
//     product of butterfly stages, grouped into `cts_levels` sparse
//     matrices with at most 2^(r+1) - 1 diagonals, each applied by
//     baby-step giant-step rotations and plaintext products; the slots then
//     hold (t_lo + i t_hi) / (2 q0 (K+1));
//  3. split real and imaginary parts with one conjugation;
//  4. EvalMod on both halves at once, in exponential form:
//     z = exp(2 pi i (K+1) u / 2^r) from two Chebyshev approximations
//     (cosine and sine parts, one shared basis), then r squarings give
//     exp(2 pi i t / q0); a squaring of a unit-modulus value only doubles
//     its error, where the double-angle formula for the cosine multiplies
//     it by up to 4 per step;
//  5. harmonic correction: with x = 2 pi t / q0, z (8 - z) = 8 e^(ix) -
//     e^(2ix), whose imaginary part 8 sin x - sin 2x = 6 x + O(x^5) has no
//     cubic term (one level), so the message may sit at q0 / 2^9 instead of
//     the q0 / 2^13 that the cubic error of sin x alone would demand;
//  6. V - conj(V) = 2 i Im V: one conjugation of the recombined halves, then
//     SlotToCoeff (the forward butterfly stages) with the factor
//     q0 / (24 pi Delta) folded into its first matrix.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <map>
#include <set>

#include <quadmath.h>

#include "host.h"
#include "poly.h"
#include "softmax.h"

namespace hs {

typedef std::complex<double> cd;
typedef std::map<int, std::vector<cd>> Mat;   // offset (mod n) -> diagonal

static void stage_exps(int N, int length, std::vector<int>& e) {
    const int h = length / 2;
    const long long lq = 4LL * length;
    e.resize(h);
    long long p = 1;
    for (int j = 0; j < h; j++) {
        e[j] = (int)(p * (2LL * N / lq));
        p = p * 5 % lq;
    }
}

// one inverse butterfly stage (a, b) -> (a + b, (a - b) conj(W_j)) on blocks of `len`
static Mat stage_inverse(const Context& c, int n, int len) {
    std::vector<int> e;
    stage_exps(c.N, len, e);
    const int h = len / 2;
    std::vector<cd> d0(n), dp(n), dm(n);
    for (int i = 0; i < n; i++) {
        const int r = i % len;
        if (r < h) {
            d0[i] = 1.0;
            dp[i] = 1.0;
        } else {
            const int j = r - h;
            const cd cw(c.tw_cos[e[j]], -c.tw_sin[e[j]]);
            d0[i] = -cw;
            dm[i] = cw;
        }
    }
    // +h and -h coincide when h = n/2: the two diagonals add
    Mat m;
    m[0] = d0;
    m[h % n] = dp;
    auto& dmr = m[(n - h) % n];
    if (dmr.empty()) dmr = dm;
    else
        for (int i = 0; i < n; i++) dmr[i] += dm[i];
    return m;
}

// one forward butterfly stage (a, b) -> (a + W_j b, a - W_j b)
static Mat stage_forward(const Context& c, int n, int len) {
    std::vector<int> e;
    stage_exps(c.N, len, e);
    const int h = len / 2;
    std::vector<cd> d0(n), dp(n), dm(n);
    for (int i = 0; i < n; i++) {
        const int r = i % len;
        if (r < h) {
            const cd w(c.tw_cos[e[r]], c.tw_sin[e[r]]);
            d0[i] = 1.0;
            dp[i] = w;
        } else {
            const cd w(c.tw_cos[e[r - h]], c.tw_sin[e[r - h]]);
            dm[i] = 1.0;
            d0[i] = -w;
        }
    }
    // +h and -h coincide when h = n/2: the two diagonals add
    Mat m;
    m[0] = d0;
    m[h % n] = dp;
    auto& dmr = m[(n - h) % n];
    if (dmr.empty()) dmr = dm;
    else
        for (int i = 0; i < n; i++) dmr[i] += dm[i];
    return m;
}

// (A B)_{da+db}[i] = sum A_da[i] B_db[i + da]  (B applied first)
static Mat mat_mul(const Mat& A, const Mat& B, int n) {
    Mat C;
    for (auto& a : A)
        for (auto& b : B) {
            const int d = (a.first + b.first) % n;
            auto& out = C[d];
            if (out.empty()) out.assign(n, 0.0);
            for (int i = 0; i < n; i++) out[i] += a.second[i] * b.second[(i + a.first) % n];
        }
    return C;
}

struct LinLevel {
    int level = 0;        // level of the input ciphertext
    int unit = 1, n1 = 1;
    double in_scale = 1, pt_scale = 1;
    std::map<int, std::vector<int>> by_giant;      // g -> babies b
    std::map<std::pair<int, int>, u64*> pt;        // (g, b) -> rows [level+1][N]
    std::vector<int> rotations() const {
        std::vector<int> r;
        std::set<int> babies;
        for (auto& kv : by_giant) {
            for (int b : kv.second) babies.insert(b);
            if (kv.first != 0) r.push_back(kv.first * n1 * unit);
        }
        for (int b : babies)
            if (b) r.push_back(b * unit);
        return r;
    }
};

struct BootCtx {
    std::vector<LinLevel> cts, stc;
    std::vector<Mat> stc_mats;     // unencoded (scales known at first use)
    std::vector<int> stc_units;
    double stc_in_scale = 0;       // scale the StC plaintexts were made for
    std::map<int, LinLevel> stc_masked;  // L -> last StC level times the 0/1 mask of slots [0, L)
    ChebPoly pcos, psin;          // cos / sin (2 pi (K+1) u / 2^r) on [-1, 1]
    double s0 = 1;                 // declared scale after ModRaise
    bool keys_done = false;
};


bool can_bootstrap(const Context& c) { return c.prm.boot.cts_levels > 0; }

// split `nst` stages into `g` groups, larger groups first
static std::vector<int> group_sizes(int nst, int g) {
    std::vector<int> s(g, nst / g);
    for (int i = 0; i < nst % g; i++) s[i]++;
    return s;
}

static void encode_level(Context& c, LinLevel& lv, const Mat& M, double constant) {
    const int n = c.N / 2;
    // split offsets t u = g n1 u + b u, pre-rotate by -g n1 u
    std::map<std::pair<int, int>, std::vector<cd>> pre;
    for (auto& kv : M) {
        double mx = 0;
        for (auto& v : kv.second) mx = std::max(mx, std::abs(v));
        if (mx < 1e-300) continue;
        const int sgn = kv.first <= n / 2 ? kv.first : kv.first - n;
        HS_REQUIRE(sgn % lv.unit == 0, E_PARAM, "linear transform: offset not a multiple of the unit");
        const int t = sgn / lv.unit;
        const int b = ((t % lv.n1) + lv.n1) % lv.n1;
        const int g = (t - b) / lv.n1;
        const int shift = ((g * lv.n1 * lv.unit) % n + n) % n;
        std::vector<cd> d(n);
        for (int i = 0; i < n; i++) d[i] = kv.second[(i - shift + n) % n] * constant;
        pre[{g, b}] = d;
        lv.by_giant[g].push_back(b);
    }
    const int rows = lv.level + 1;
    std::vector<double> re(n), im(n), w(c.N);
    double* dw = (double*)c.pool.alloc(sizeof(double) * c.N);
    for (auto& kv : pre) {
        for (int i = 0; i < n; i++) {
            re[i] = kv.second[i].real();
            im[i] = kv.second[i].imag();
        }
        special_fft_inverse(c, re, im);
        for (int k = 0; k < n; k++) {
            w[k] = re[k];
            w[k + n] = im[k];
        }
        c.upload(dw, w.data(), sizeof(double) * c.N);
        u64* pt = (u64*)c.persistent_alloc(sizeof(u64) * rows * c.N, "bootstrap plaintexts");
        Rows r = c.rows(pt, 1, rows, (size_t)rows * c.N);
        k_encode_real(c.T, r, dw, 0, lv.pt_scale, c.stream);
        k_ntt(c.T, r, false, c.stream);
        lv.pt[kv.first] = pt;
    }
    c.sync();
    c.pool.free(dw);
}

// per-context tables (no global state: contexts on different host threads
// bootstrap independently)
static BootCtx& boot_ctx(Context& c) {
    if (c.boot) return *(BootCtx*)c.boot;
    HS_REQUIRE(can_bootstrap(c), E_PARAM, "no bootstrapping parameters");
    const BootParams& bp = c.prm.boot;
    HS_REQUIRE(c.prm.user_top + bp.cts_levels + bp.evalmod_levels + bp.stc_levels == c.L, E_PARAM,
               "bootstrapping levels do not match the modulus chain");
    HS_REQUIRE(cheb_depth(bp.cos_degree) + bp.double_angle + 1 == bp.evalmod_levels, E_PARAM,
               "EvalMod levels must be the polynomial depth + squarings + 1");
    BootCtx* B = new BootCtx();
    const int n = c.N / 2;
    int nst = 0;
    while ((1 << nst) < n) nst++;
    const double q0 = (double)c.primes[0];
    const double Db = std::ldexp(1.0, bp.log_boot_scale);
    // ---- CoeffToSlot: stages of length n, n/2, ..., 2 (in application order)
    {
        std::vector<int> gs = group_sizes(nst, bp.cts_levels);
        B->s0 = 2.0 * q0 * (bp.K + 1) * n;
        int len = n;
        double s_prev = B->s0;
        for (int gi = 0; gi < bp.cts_levels; gi++) {
            Mat M;
            bool first = true;
            int unit = len;
            for (int s = 0; s < gs[gi]; s++) {
                Mat S = stage_inverse(c, n, len);
                M = first ? S : mat_mul(S, M, n);
                first = false;
                unit = len / 2;
                len /= 2;
            }
            LinLevel lv;
            lv.level = c.L - gi;
            lv.unit = unit;
            lv.n1 = 1 << ((gs[gi] + 1) / 2);
            const double frac = (double)(gi + 1) / bp.cts_levels;
            const double s_next = std::exp2(std::log2(B->s0) * (1 - frac) + std::log2(Db) * frac);
            lv.in_scale = s_prev;
            lv.pt_scale = s_next * (double)c.primes[lv.level] / s_prev;
            encode_level(c, lv, M, 1.0);
            s_prev = s_prev * lv.pt_scale / (double)c.primes[lv.level];
            B->cts.push_back(lv);
        }
    }
    // ---- SlotToCoeff: stages of length 2, 4, ..., n; encoded at first use
    {
        std::vector<int> gs = group_sizes(nst, bp.stc_levels);
        std::reverse(gs.begin(), gs.end());
        int len = 2;
        for (int gi = 0; gi < bp.stc_levels; gi++) {
            Mat M;
            bool first = true;
            int unit = len / 2;
            for (int s = 0; s < gs[gi]; s++) {
                Mat S = stage_forward(c, n, len);
                M = first ? S : mat_mul(S, M, n);
                first = false;
                len *= 2;
            }
            B->stc_mats.push_back(M);
            B->stc_units.push_back(unit);
            LinLevel lv;
            lv.level = c.prm.user_top + bp.stc_levels - gi;
            lv.unit = unit;
            lv.n1 = 1 << ((gs[gi] + 1) / 2);
            // register the rotation layout now (plaintexts later)
            const int nn = n;
            for (auto& kv : M) {
                const int sgn = kv.first <= nn / 2 ? kv.first : kv.first - nn;
                const int t = sgn / unit;
                const int b = ((t % lv.n1) + lv.n1) % lv.n1;
                lv.by_giant[(t - b) / lv.n1].push_back(b);
            }
            B->stc.push_back(lv);
        }
    }
    // ---- EvalMod polynomials (parity enforced: cos is even, sin is odd)
    {
        const quad w = 2 * M_PIq * (bp.K + 1) * ldexpq(1, -bp.double_angle);
        B->pcos = cheb_fit([&](quad u) { return cosq(w * u); }, -1.0, 1.0, bp.cos_degree);
        B->psin = cheb_fit([&](quad u) { return sinq(w * u); }, -1.0, 1.0, bp.cos_degree);
        for (size_t j = 0; j < B->pcos.c.size(); j++) (j % 2 ? B->pcos.c[j] : B->psin.c[j]) = 0.0;
    }
    c.boot = B;
    return *B;
}

static void ensure_keys(Context& c, BootCtx& B) {
    if (B.keys_done) return;
    add_galois_key(c, 2 * c.N - 1);
    for (auto* levels : {&B.cts, &B.stc})
        for (auto& lv : *levels)
            for (int r : lv.rotations()) add_galois_key(c, galois_rot(r, c.N));
    B.keys_done = true;
}

// baby-step giant-step application of one encoded level; one rescale
// (skipped when do_rescale is false: the caller rescales later)
static Ct apply_level(Context& c, const LinLevel& lv, const Ct& x, bool do_rescale = true) {
    HS_REQUIRE(x.level == lv.level, E_LEVEL, "linear transform: unexpected input level");
    const size_t cw = x.ct_words(c.N) * x.m;   // words of one rotation of x
    // baby steps: every nonzero rotation of x in one hoisted batch
    std::set<int> need;
    for (auto& kv : lv.by_giant)
        for (int b : kv.second)
            if (b != 0) need.insert(b);
    std::map<int, int> slot;
    Ct babies;
    if (!need.empty()) {
        std::vector<int> rs;
        for (int b : need) {
            slot[b] = (int)rs.size();
            rs.push_back(b * lv.unit);
        }
        babies = op_rotate_hoisted_batch(c, x, rs);
    }
    auto baby = [&](int b) -> const u64* { return b == 0 ? x.d : babies.d + (size_t)slot.at(b) * cw; };
    // sums over the babies of baby_b * diag_(g,b) (one fused launch per giant
    // step): giant 0 straight into the accumulator, the others into one batch
    // that takes all its giant-step rotations in one batched key switch
    Ct acc = ct_alloc(c, x.m, 2, x.level);
    acc.scale = x.scale * lv.pt_scale;
    std::vector<int> giants;
    for (auto& kv : lv.by_giant)
        if (kv.first != 0) giants.push_back(kv.first);
    Ct inner;
    if (!giants.empty()) {
        inner = ct_alloc(c, (int)giants.size() * x.m, 2, x.level);
        inner.scale = acc.scale;
    }
    bool have0 = false;
    int gi = 0;
    for (auto& kv : lv.by_giant) {
        std::vector<const u64*> as, ps;
        for (int b : kv.second) {
            as.push_back(baby(b));
            ps.push_back(lv.pt.at({kv.first, b}));
        }
        u64* dst = kv.first == 0 ? acc.d : inner.d + (size_t)(gi++) * cw;
        if (kv.first == 0) have0 = true;
        c.count(OC_PTMUL, x.level, (double)x.m * as.size());
        c.count(OC_ADD, x.level, (double)x.m * (as.size() - 1));
        k_mul_plain_acc(c.T, dst, as.data(), ps.data(), (int)as.size(), x.m * 2, x.level + 1, c.stream);
    }
    if (babies.d) ct_free(c, babies);
    if (!giants.empty()) {
        std::vector<int> gal;
        for (int g : giants) gal.push_back(galois_rot(g * lv.n1 * lv.unit, c.N));
        Ct rot = op_galois_batch(c, inner, gal, x.m);
        ct_free(c, inner);
        const Rows ra = c.ct_rows(acc);
        for (size_t i = 0; i < giants.size(); i++) {
            Rows rr = ra;
            rr.base = rot.d + i * cw;
            if (i == 0 && !have0) {
                k_copy_rows(c.T, ra, rr, c.stream);
            } else {
                c.count(OC_ADD, acc.level, acc.m);
                k_add(c.T, ra, ra, rr, c.stream);
            }
        }
        ct_free(c, rot);
    }
    if (!do_rescale) return acc;
    Ct out = op_rescale(c, acc);
    ct_free(c, acc);
    return out;
}

// SlotToCoeff plaintexts, encoded once for the EvalMod output scale of an
// unscaled message (`in_scale`); apply_level tracks the actual scale.
static void encode_stc(Context& c, BootCtx& B, double in_scale) {
    if (B.stc_in_scale != 0) {
        HS_REQUIRE(std::fabs(B.stc_in_scale / in_scale - 1.0) < 1e-9, E_STATE,
                   "bootstrapping: EvalMod output scale changed");
        return;
    }
    const BootParams& bp = c.prm.boot;
    const double q0 = (double)c.primes[0];
    const double Dout = std::ldexp(1.0, c.prm.log_scale);
    const double two_pi = 6.283185307179586;
    const double cst = q0 / (12.0 * two_pi * Dout);   // the input holds 2 (8 sin x - sin 2x), x = 2 pi t / q0
    double s_prev = in_scale;
    for (int gi = 0; gi < bp.stc_levels; gi++) {
        LinLevel& lv = B.stc[gi];
        lv.by_giant.clear();
        const double frac = (double)(gi + 1) / bp.stc_levels;
        const double s_next = std::exp2(std::log2(in_scale) * (1 - frac) + std::log2(Dout) * frac);
        lv.in_scale = s_prev;
        lv.pt_scale = s_next * (double)c.primes[lv.level] / s_prev;
        encode_level(c, lv, B.stc_mats[gi], gi == 0 ? cst : 1.0);
        s_prev = s_prev * lv.pt_scale / (double)c.primes[lv.level];
    }
    B.stc_in_scale = in_scale;
}

// The last SlotToCoeff level with the slot mask [0, L) folded into its
// diagonals: diag(mask) sum_k diag(d_k) rot_k = sum_k diag(mask d_k) rot_k,
// so the output is the refreshed value on slots [0, L) and exactly zero (up
// to the rescaling error) elsewhere, at no extra level.
static const LinLevel& stc_masked_level(Context& c, BootCtx& B, int L) {
    auto it = B.stc_masked.find(L);
    if (it != B.stc_masked.end()) return it->second;
    const int n = c.N / 2;
    HS_REQUIRE(L >= 1 && L <= n, E_ARG, "bootstrap: mask length out of range");
    HS_REQUIRE(B.stc_in_scale != 0, E_STATE, "bootstrap: SlotToCoeff not encoded");
    const LinLevel& base = B.stc.back();
    LinLevel lv;
    lv.level = base.level;
    lv.unit = base.unit;
    lv.n1 = base.n1;
    lv.in_scale = base.in_scale;
    lv.pt_scale = base.pt_scale;
    Mat M = B.stc_mats.back();
    for (auto& kv : M)
        for (int i = L; i < n; i++) kv.second[i] = 0.0;
    double constant = 1.0;
    if (B.stc.size() == 1) {
        const double two_pi = 6.283185307179586;
        constant = (double)c.primes[0] / (12.0 * two_pi * std::ldexp(1.0, c.prm.log_scale));
    }
    encode_level(c, lv, M, constant);
    return B.stc_masked.emplace(L, lv).first->second;
}

// Large batches are refreshed 16 ciphertexts at a time: every step acts per
// ciphertext, and the transient memory of a bootstrap (hoisted key-switching
// buffers and baby-step rotations at the top level, ~1 GB per ciphertext at
// N = 2^16) would otherwise grow with the batch.
Ct bootstrap(Context& c, const Ct& x, double bound, int mask_L) {
    constexpr int kChunk = 16;
    if (x.m <= kChunk) return bootstrap_stage(c, x, bound, 0, mask_L);
    std::vector<Ct> parts;
    for (int i = 0; i < x.m; i += kChunk) {
        Ct in = ct_slice(c, x, i, std::min(kChunk, x.m - i));
        parts.push_back(bootstrap_stage(c, in, bound, 0, mask_L));
        ct_free(c, in);
    }
    std::vector<const Ct*> ptrs;
    for (auto& q : parts) ptrs.push_back(&q);
    Ct out = ct_gather(c, ptrs);
    for (auto& q : parts) ct_free(c, q);
    return out;
}

// stop: 0 = full; 1 = after ModRaise; 2 = after CoeffToSlot; 3 = real part
// after the split; 4 = real-part half of z after the polynomials; 5 / 6 =
// real / imaginary half of z after the squarings; 7 = SlotToCoeff input;
// 8, 9 = after the first SlotToCoeff levels (intermediate results for tests)
Ct bootstrap_stage(Context& c, const Ct& x, double bound, int stop, int mask_L) {
    HS_REQUIRE(can_bootstrap(c), E_PARAM, "no bootstrapping parameters");
    HS_REQUIRE(x.ncomp == 2, E_ARG, "bootstrap: degree-1 ciphertext expected");
    BootCtx& B = boot_ctx(c);
    ensure_keys(c, B);
    const BootParams& bp = c.prm.boot;
    const double q0 = (double)c.primes[0];
    const double Db = std::ldexp(1.0, bp.log_boot_scale);
    const double Bd = std::max(bound, std::ldexp(1.0, -20));
    // 1. message size |m| ~ q0 / 2^9 at the bound
    const double target = q0 / 512.0;
    Ct xx;
    int e = 0;
    double kfac = 1.0;   // integer factor the message was scaled up by
    if (Bd * x.scale > 2.0 * target && x.level >= 1) {
        e = (int)std::ceil(std::log2(Bd * x.scale / target));
        xx = op_mul_const(c, x, std::ldexp(1.0, -e), x.scale);
    } else {
        xx = ct_copy(c, x);
        // at most 16: the factor is undone inside EvalMod (below), which
        // lowers the SlotToCoeff scales by the same factor
        const double kf = std::min(std::floor(target / (Bd * x.scale)), 16.0);
        if (kf >= 2.0) {
            const long long K = (long long)kf;
            op_mul_int_inplace(c, xx, K);
            xx.scale = x.scale * (double)K;
            kfac = (double)K;
        }
    }
    const double s_msg = xx.scale;
    Ct x0 = ct_drop(c, xx, 0);
    ct_free(c, xx);
    Ct t = op_mod_raise(c, x0, c.L);
    ct_free(c, x0);
    t.scale = B.s0;
    if (stop == 1) return t;
    // 2. CoeffToSlot; the last level is left unrescaled so that the
    // conjugation's key-switching noise is added at scale s * pt_scale and
    // vanishes in the rescale (it is the largest noise of the pipeline
    // otherwise: it reaches the output amplified by sqrt(N/2) (K+1) 2^14)
    for (size_t li = 0; li < B.cts.size(); li++) {
        const bool last = li + 1 == B.cts.size();
        Ct nx = apply_level(c, B.cts[li], t, !last);
        ct_free(c, t);
        t = nx;
    }
    // 3. real / imaginary split: u_re = t + conj t, u_im = -i (t - conj t)
    Ct cj = op_conjugate(c, t);
    Ct ure = op_add(c, t, cj);
    Ct dif = op_sub(c, t, cj);
    Ct uim = op_mul_monomial(c, dif, 3 * c.N / 2);
    ct_free(c, dif);
    ct_free(c, cj);
    if (stop == 2) {
        ct_free(c, ure);
        ct_free(c, uim);
        Ct r = op_rescale(c, t);
        ct_free(c, t);
        return r;
    }
    ct_free(c, t);
    std::vector<const Ct*> parts{&ure, &uim};
    Ct ug = ct_gather(c, parts);
    const int m = x.m;
    ct_free(c, ure);
    ct_free(c, uim);
    Ct u = op_rescale(c, ug);
    ct_free(c, ug);
    if (stop == 3) {
        Ct r = ct_slice(c, u, 0, m);
        ct_free(c, u);
        return r;
    }
    // 4. EvalMod: z = exp(2 pi i (K+1) u / 2^r), then r squarings.  The
    // polynomial's output scale Db kfac^(-2^-(r+1)) becomes, after the r
    // squarings and the product of step 5, a physical scale kfac times
    // lower than for kfac = 1: the SlotToCoeff output then carries the
    // message at the input's scale instead of kfac times it.
    Ct z;
    {
        const double Dp = Db * std::pow(kfac, -std::ldexp(1.0, -(bp.double_angle + 1)));
        // cos + i sin as one polynomial with complex coefficients
        z = eval_cheb_complex(c, u, B.pcos, B.psin, Dp);
        ct_free(c, u);
    }
    if (stop == 4) {
        Ct r = ct_slice(c, z, 0, m);
        ct_free(c, z);
        return r;
    }
    for (int r = 0; r < bp.double_angle; r++) {
        Ct s = op_mult(c, z, z);
        ct_free(c, z);
        z = s;
    }
    if (stop == 5 || stop == 6) {
        Ct r = ct_slice(c, z, stop == 5 ? 0 : m, m);
        ct_free(c, z);
        return r;
    }
    // 5. V = z (8 - z)
    {
        Ct w = ct_copy(c, z);
        op_neg_inplace(c, w);
        op_add_const_inplace(c, w, 8.0);
        Ct v = op_mult(c, z, w);
        ct_free(c, w);
        ct_free(c, z);
        z = v;
    }
    // 6. y = 2 (Im V_re + i Im V_im) = A - conj(B) with
    //    A = -i V_re + V_im and B = i V_re + V_im
    Ct zre = ct_slice(c, z, 0, m);
    Ct zim = ct_slice(c, z, m, m);
    ct_free(c, z);
    Ct A = op_mul_monomial(c, zre, 3 * c.N / 2);
    op_add_inplace(c, A, zim);
    Ct Bp = op_mul_monomial(c, zre, c.N / 2);
    op_add_inplace(c, Bp, zim);
    ct_free(c, zre);
    ct_free(c, zim);
    Ct cB = op_conjugate(c, Bp);
    ct_free(c, Bp);
    Ct vre = op_sub(c, A, cB);
    ct_free(c, A);
    ct_free(c, cB);
    encode_stc(c, B, vre.scale * kfac);
    Ct y = vre;
    if (stop == 7) return y;
    const LinLevel* last_masked = mask_L > 0 ? &stc_masked_level(c, B, mask_L) : nullptr;
    int lvl_i = 0;
    for (size_t gi = 0; gi < B.stc.size(); gi++) {
        const LinLevel& lv = (last_masked && gi + 1 == B.stc.size()) ? *last_masked : B.stc[gi];
        Ct ny = apply_level(c, lv, y);
        ct_free(c, y);
        y = ny;
        lvl_i++;
        if (stop == 7 + lvl_i) return y;
    }
    // the StC output encodes v * s_msg / Delta at its computed scale
    const double Dout = std::ldexp(1.0, c.prm.log_scale);
    y.scale = y.scale * s_msg / Dout;
    if (e > 0) {
        op_mul_int_inplace(c, y, 1LL << e);
    }
    return y;
}

void boot_release(Context* c) {
    delete (BootCtx*)c->boot;
    c->boot = nullptr;
}

}  // namespace hs
