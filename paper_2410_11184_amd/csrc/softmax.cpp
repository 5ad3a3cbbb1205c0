// Homomorphic Softmax by normalize-and-square.
//
//  * Algorithm SM (Section 3.2): y0 = exp(x / 2^k); for j = 1..k:
//    lambda_j = (sum_i y_i^2)^(-1/2), z = lambda_j y, y = z^2.
//  * The auxiliary thread (Algorithm "alg:AuxThread", Section 3.3): square,
//    rotate-and-add with strides -L 2^t, the normalisation polynomial, mask
//    to slots [0, L), rotate-and-add with strides +L 2^t.
//  * Many ciphertexts (Section 4.2): m ciphertexts hold L = m N0 / n Softmax;
//    the squares of all m are summed into one auxiliary ciphertext before the
//    log2(n/m) rotations, and one auxiliary thread serves all of them.
//  * Version B (Algorithm "alg:Softmax1B", Section 4.3): lambda_j =
//    (sum y^(j-1)^2)^(-2^-j), Lambda *= lambda_j, z = Lambda y0,
//    y^(j) = z^(2^j), so the main thread spends one level per iteration plus
//    the squarings.  Its last iteration is evaluated as one normalize-and-
//    square step on y^(k-1), y^(k) = (S_k^(-1/2) y^(k-1))^2, which is the same
//    value (Lambda_k^(2^k) y0^(2^k) = y^(k-1)^2 / S_k) with two main-thread
//    levels and an error that is not amplified by 2^k.
//  * Bootstraps follow the rules of Section 5.1 ("Bootstrapping strategy in
//    the many ciphertexts case"): bootstrap the auxiliary ciphertext before
//    the normalisation polynomial when its budget is short, again afterwards
//    if its level is below what the main thread needs, and the main thread
//    only when its own budget runs out.  The normalisation factors (lambda_j,
//    and Lambda in version B) are bootstrapped while they sit on slots
//    [0, L) only, with the mask folded into the bootstrap, and broadcast
//    afterwards: the bootstrapping error is then one value per Softmax, a
//    common factor that the next renormalisation removes, instead of an
//    independent error per element that the squarings amplify by 2^k.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include <quadmath.h>

#include "host.h"
#include "poly.h"
#include "softmax.h"

namespace hs {

// device coefficients of the 0/1 slot vector with ones on slots [lo, hi)
static const double* mask_coeffs(Context& c, int lo, int hi) {
    const int n = c.N / 2;
    const int key = lo * (n + 1) + hi;
    auto it = c.mask_coeffs.find(key);
    if (it != c.mask_coeffs.end()) return it->second;
    std::vector<double> re(n, 0.0), im(n, 0.0);
    for (int j = lo; j < hi; j++) re[j] = 1.0;
    special_fft_inverse(c, re, im);
    std::vector<double> w(c.N);
    for (int k = 0; k < n; k++) {
        w[k] = re[k];
        w[k + n] = im[k];
    }
    double* d = (double*)c.dev_table(w.data(), sizeof(double) * c.N);
    c.mask_coeffs[key] = d;
    return d;
}

static const double* mask_coeffs(Context& c, int L) { return mask_coeffs(c, 0, L); }

int theorem_k(int n, double M) {
    const double v = std::ceil(std::log2(M) - std::log2(std::log((double)n)));
    return std::max(1, (int)v);
}

// iterations of the t-th power variant: M / t^k ~ ln n (the appendix on other
// normalisations); t = 2 is the Theorem's k
static int power_k(int n, double M, int t) {
    if (t == 2) return theorem_k(n, M);
    const double v = std::ceil((std::log2(M) - std::log2(std::log((double)n))) / std::log2((double)t));
    return std::max(1, (int)v);
}

// y^t for t in {2, 3, 4} (ceil(log2 t) levels)
static Ct op_power(Context& c, const Ct& y, int t) {
    Ct y2 = op_mult(c, y, y);
    if (t == 2) return y2;
    Ct o = op_mult(c, y2, t == 3 ? y : y2);
    ct_free(c, y2);
    return o;
}

// per job, the sum of its m ciphertexts (a.m = jobs m)
static Ct op_sum_jobs(Context& c, const Ct& a, int jobs) {
    const int m = a.m / jobs;
    Ct o = ct_alloc(c, jobs, a.ncomp, a.level);
    o.scale = a.scale;
    const size_t w = a.ct_words(c.N);
    const int rows = a.ncomp * (a.level + 1);
    for (int j = 0; j < jobs; j++) {
        Rows dst{o.d + (size_t)j * w, 1, rows, w, a.level + 1, 0, c.nq};
        Rows first{a.d + (size_t)j * m * w, 1, rows, w, a.level + 1, 0, c.nq};
        k_copy_rows(c.T, dst, first, c.stream);
        for (int i = 1; i < m; i++) {
            Rows src{a.d + (size_t)(j * m + i) * w, 1, rows, w, a.level + 1, 0, c.nq};
            c.count(OC_ADD, a.level, a.ncomp / 2.0);
            k_add(c.T, dst, dst, src, c.stream);
        }
    }
    return o;
}

static int ilog2(int x) {
    int l = 0;
    while ((1 << l) < x) l++;
    return l;
}

// max over a dense grid of |p(s) s^e - 1| on [lo, hi]
static double rel_error(const ChebPoly& p, double lo, double hi, double e) {
    double worst = 0;
    const int G = 4000;
    for (int i = 0; i <= G; i++) {
        // geometric grid (the error is largest near the lower end)
        const double s = lo * std::pow(hi / lo, (double)i / G);
        worst = std::max(worst, std::fabs(cheb_eval_plain(p, s) * std::pow(s, e) - 1.0));
    }
    return worst;
}

static double max_abs(const ChebPoly& p, double lo, double hi) {
    double m = 0;
    for (int i = 0; i <= 2000; i++) m = std::max(m, std::fabs(cheb_eval_plain(p, lo + (hi - lo) * i / 2000.0)));
    return m;
}

// Chebyshev interval [a, a + 2^e] covering [lo, hi] with 2^e <= 2 (so the
// affine map to [-1, 1] is an integer product and a constant addition)
static void free_interval(double lo, double hi, double& a, double& b) {
    a = lo;
    double w = 1.0;
    while (w < hi - lo) w *= 2;
    while (w / 2 >= hi - lo && w > 1.0 / 64) w /= 2;
    b = a + w;
}

// bound on |Lambda| for its bootstrapping: Lambda_j ~ 1 / ||y0||_(2^(j+1))
// stays below sqrt(n) for rows whose largest logit is near 0; a loose bound
// costs little since Lambda's bootstrapping error is one factor per Softmax
static double lam_bound_big(int n, double lam_bound) {
    return std::max({64.0, lam_bound, 4.0 * std::sqrt((double)n)});
}

// Bootstrap x when its level is below `need`.  mask_L > 0: x is zero off
// slots [0, L) and the refreshed value is masked the same way, so that its
// bootstrapping error, once broadcast, is the same for every element of a
// Softmax and is removed by the next renormalisation.
// HS_TRACE >= 2 (eager runs only): decrypt a bootstrapping's input and
// output (first ciphertext) and print the largest slot difference, absolute
// and relative to the input's largest slot (masked: slots [0, L) against the
// input, the rest against zero)
static void trace_boot_error(Context& c, const Ct& x, const Ct& b, int mask_L) {
    const int n = c.N / 2;
    std::vector<double> xr(n), xi(n), br(n), bi(n);
    decrypt_decode(c, x, 0, xr.data(), xi.data());
    decrypt_decode(c, b, 0, br.data(), bi.data());
    double err = 0, big = 0, small = 1e300;
    for (int k = 0; k < n; k++) {
        const bool keep = mask_L <= 0 || k < mask_L;
        const double wr = keep ? xr[k] : 0.0, wi = keep ? xi[k] : 0.0;
        err = std::max(err, std::hypot(br[k] - wr, bi[k] - wi));
        big = std::max(big, std::fabs(wr));
        if (keep) small = std::min(small, std::fabs(wr));
    }
    std::fprintf(stderr, "[hs]   bootstrap error 2^%.2f (input |x| in [%.3g, %.3g], level %d, scale 2^%.2f)\n",
                 std::log2(err + 1e-300), small, big, x.level, std::log2(x.scale));
}

static Ct ensure_level(Context& c, const Ct& x, int need, double bound, SoftmaxStats& st, bool& replaced,
                       const char* what, int iter, int mask_L = 0) {
    replaced = false;
    if (x.level >= need) return x;
    HS_REQUIRE(can_bootstrap(c), E_LEVEL, "Softmax: level budget exhausted and no bootstrapping configured");
    if (std::getenv("HS_TRACE"))
        std::fprintf(stderr, "[hs] softmax iteration %d: bootstrap %s (%d ct, level %d -> need %d, bound %g%s)\n",
                     iter, what, x.m, x.level, need, bound, mask_L ? ", masked" : "");
    Ct b = bootstrap(c, x, bound, mask_L);
    st.bootstraps += x.m;
    replaced = true;
    const char* tr = std::getenv("HS_TRACE");
    if (tr && std::atoi(tr) >= 2 && !c.capturing) trace_boot_error(c, x, b, mask_L);
    HS_REQUIRE(b.level >= need, E_LEVEL, "Softmax: bootstrapping does not restore enough levels");
    return b;
}

// Padded dimension (n below the power of two np2 it is packed in): y0 times
// the 0/1 indicator of the real coordinates.  Ciphertext j of a job holds
// coordinates j per .. (j + 1) per - 1 on slot blocks of L, so its indicator
// keeps slots [0, R_j), R_j = (n - j per) L clamped to [0, N/2]: a plaintext
// product at scale q_l and one rescale (scale unchanged).
static Ct mask_padding(Context& c, const Ct& y0, int n, int per, int L, int m) {
    const int N0 = c.N / 2;
    const int lv = y0.level;
    HS_REQUIRE(lv >= 1, E_LEVEL, "Softmax: no level for the padding mask");
    const double ql = (double)c.primes[lv];
    Ct o = ct_alloc(c, y0.m, 2, lv);
    o.scale = y0.scale * ql;
    const size_t cw = y0.ct_words(c.N), pw = y0.comp_words(c.N);
    for (int g = 0; g < y0.m; g++) {
        const long long R = std::min<long long>(std::max<long long>((long long)(n - (g % m) * per) * L, 0), N0);
        bool owned;
        u64* pt = mask_plaintext(c, mask_coeffs(c, (int)R), lv, ql, &owned);
        Rows ra{y0.d + (size_t)g * cw, 2, lv + 1, pw, lv + 1, 0, c.nq};
        Rows ro{o.d + (size_t)g * cw, 2, lv + 1, pw, lv + 1, 0, c.nq};
        Rows rp{pt, 2, lv + 1, 0, lv + 1, 0, c.nq};
        c.count(OC_PTMUL, lv, 1.0);
        k_mul(c.T, ro, ra, rp, c.stream);
        if (owned) c.free_words(pt);
    }
    Ct r = op_rescale(c, o);
    ct_free(c, o);
    r.scale = y0.scale;
    return r;
}

// Inverse square root by Newton's iteration (Appendix A, the lemma on
// computing inverse square roots): from the first guess y ~ S^(-1/2),
// `steps` times y <- 3/2 y - (S/2 y)(y y), two levels per step.  Every step
// lands at scale tgt exactly, as the polynomial evaluator's results do: S/2
// is taken by a constant product at the scale T1 that makes (S/2 y)(y y)
// come out at tgt, and 3/2 y by a constant product at tgt (S has levels
// above y, so S/2 costs none of y's).  The last step also applies the mask
// (`mask` given: S/2 and 3/2 y as masked plaintext products) or the
// averaging factor 1/avg (in both constants).
static Ct newton_invsqrt(Context& c, const Ct& S, const Ct& y0, int steps, const double* mask, int avg,
                         double tgt) {
    Ct y = ct_copy(c, y0);
    for (int i = 0; i < steps; i++) {
        const bool lastn = i + 1 == steps;
        const int l = y.level;
        HS_REQUIRE(l >= 2 && S.level > l, E_LEVEL, "Newton step: levels");
        const double ql = (double)c.primes[l], ql1 = (double)c.primes[l - 1];
        const double T1 = tgt * ql * ql * ql1 / (y.scale * y.scale * y.scale);
        Ct h;
        if (lastn && mask) {
            const double qs = (double)c.primes[S.level];
            const double ps = T1 * qs / S.scale;
            bool owned;
            u64* pt = mask_plaintext(c, mask, S.level, 0.5 * ps, &owned);
            h = op_mul_plain(c, S, pt, ps, true);
            if (owned) c.free_words(pt);
            h.scale = T1;
        } else {
            h = op_mul_const(c, S, lastn ? 0.5 / avg : 0.5, T1);
        }
        Ct z1 = op_mult(c, h, y);
        ct_free(c, h);
        Ct z2 = op_mult(c, y, y);
        Ct w = op_mult(c, z1, z2);
        ct_free(c, z1);
        ct_free(c, z2);
        Ct z3;
        if (lastn && mask) {
            const double ps = tgt * ql / y.scale;
            bool owned;
            u64* pt = mask_plaintext(c, mask, l, 1.5 * ps, &owned);
            z3 = op_mul_plain(c, y, pt, ps, true);
            if (owned) c.free_words(pt);
            z3.scale = tgt;
        } else {
            z3 = op_mul_const(c, y, lastn ? 1.5 / avg : 1.5, tgt);
        }
        Ct z3d = ct_drop(c, z3, w.level);
        ct_free(c, z3);
        op_sub_inplace(c, z3d, w);
        ct_free(c, w);
        ct_free(c, y);
        y = z3d;
    }
    return y;
}

// Newton's error map for the inverse square root: y sqrt(s) = 1 + e gives
// 1 - e^2 (3 + e) / 2 after one step; a relative error bound delta becomes
// delta^2 (3 + delta) / 2
static double newton_delta(double delta, int steps) {
    for (int i = 0; i < steps; i++) delta = delta * delta * (3.0 + delta) / 2.0;
    return delta;
}

// rotate-and-add with strides +L 2^t: slots [0, L) copied to all n/m blocks
static void broadcast(Context& c, Ct& a, int L, int nrot) {
    for (int t = 0; t < nrot; t++) {
        Ct rr = op_rotate(c, a, L << t);
        op_add_inplace(c, a, rr);
        ct_free(c, rr);
    }
}

// a (one ciphertext per job) repeated m times per job, to pair with the main
// batch; a itself when there is one job (the products broadcast it)
static Ct per_job(Context& c, const Ct& a, int jobs, int m) {
    if (jobs == 1) return ct_copy(c, a);
    Ct o = ct_alloc(c, jobs * m, a.ncomp, a.level);
    o.scale = a.scale;
    const size_t w = a.ct_words(c.N);
    for (int j = 0; j < jobs; j++) {
        Rows dst{o.d + (size_t)j * m * w, m, a.ncomp * (a.level + 1), w, a.level + 1, 0, c.nq};
        Rows src{a.d + (size_t)j * w, m, a.ncomp * (a.level + 1), 0, a.level + 1, 0, c.nq};
        k_copy_rows(c.T, dst, src, c.stream);
    }
    return o;
}

// Many jobs, few auxiliary ciphertexts (Section 4.2's packing of the sums
// of many Softmax into one ciphertext, across jobs): the J jobs' sums S (one
// ciphertext per job, each holding its L sums on every block of L slots
// after the rotate-and-add) become G = J / Jg ciphertexts, the g-th holding
// job g Jg + b's sums on block b (Jg = min(J, N/2 / L) jobs each), by 0/1
// plaintexts of the blocks at scale q_l summed before one rescale (the
// scale stays S's).
static Ct pack_jobs(Context& c, const Ct& S, int L, int Jg) {
    const int J = S.m, lv = S.level, G = J / Jg;
    HS_REQUIRE(lv >= 1, E_LEVEL, "Softmax: no level to pack the jobs' auxiliary ciphertexts");
    const double ql = (double)c.primes[lv];
    Ct o = ct_alloc(c, G, 2, lv);
    o.scale = S.scale * ql;
    std::vector<u64*> own;
    for (int g = 0; g < G; g++) {
        std::vector<const u64*> as, ps;
        for (int b = 0; b < Jg; b++) {
            bool owned;
            u64* pt = mask_plaintext(c, mask_coeffs(c, b * L, (b + 1) * L), lv, ql, &owned);
            as.push_back(S.d + (size_t)(g * Jg + b) * S.ct_words(c.N));
            ps.push_back(pt);
            if (owned) own.push_back(pt);
        }
        c.count(OC_PTMUL, lv, (double)Jg);
        c.count(OC_ADD, lv, (double)(Jg - 1));
        k_mul_plain_acc(c.T, o.d + (size_t)g * o.ct_words(c.N), as.data(), ps.data(), Jg, 2, lv + 1, c.stream);
    }
    for (u64* p : own) c.free_words(p);
    Ct r = op_rescale(c, o);
    ct_free(c, o);
    r.scale = S.scale;
    return r;
}

// The inverse for factors computed on the packed ciphertexts a: job g Jg + b's
// factor is a_g times the 0/1 plaintext of block b at scale q_l, one rescale
// (the scale stays a's); J ciphertexts, job by job, each nonzero on its own
// block only, which the broadcast (its rotate-and-add runs over every block)
// copies to all blocks.
static Ct unpack_jobs(Context& c, const Ct& a, int J, int L, int Jg) {
    const int lv = a.level;
    HS_REQUIRE(lv >= 1, E_LEVEL, "Softmax: no level to take the jobs' factors apart");
    const double ql = (double)c.primes[lv];
    Ct o = ct_alloc(c, J, 2, lv);
    o.scale = a.scale * ql;
    for (int i = 0; i < J; i++) {
        const int g = i / Jg, b = i % Jg;
        bool owned;
        u64* pt = mask_plaintext(c, mask_coeffs(c, b * L, (b + 1) * L), lv, ql, &owned);
        const Rows ra{a.d + (size_t)g * a.ct_words(c.N), 2, lv + 1, a.comp_words(c.N), lv + 1, 0, c.nq};
        Rows ro{o.d + (size_t)i * o.ct_words(c.N), 2, lv + 1, o.comp_words(c.N), lv + 1, 0, c.nq};
        Rows rp{pt, 2, lv + 1, 0, lv + 1, 0, c.nq};
        c.count(OC_PTMUL, lv, 1.0);
        k_mul(c.T, ro, ra, rp, c.stream);
        if (owned) c.free_words(pt);
    }
    Ct r = op_rescale(c, o);
    ct_free(c, o);
    r.scale = a.scale;
    return r;
}

Ct softmax(Context& c, const Ct& x, int n, double M, const SoftmaxOpts& o, SoftmaxStats* stats, int jobs) {
    SoftmaxStats st;
    const int N0 = c.N / 2;
    HS_REQUIRE(jobs >= 1 && x.m % jobs == 0, E_ARG, "Softmax: batch not divisible into jobs");
    const int J = jobs;
    const int m = x.m / J;
    HS_REQUIRE(n >= 2, E_PARAM, "Softmax dimension must be >= 2");
    // a dimension that is not a power of two is packed as the next power of
    // two, its extra coordinates removed by a mask after the exponential
    const int np2 = 1 << ilog2(n);
    HS_REQUIRE(np2 <= N0 && m >= 1 && np2 % m == 0, E_ARG, "need m | n <= N/2 (n rounded up to a power of two)");
    HS_REQUIRE(M > 0, E_ARG, "range M must be positive");
    HS_REQUIRE(x.ncomp == 2, E_ARG, "degree-1 ciphertexts expected");
    const bool smb = o.variant == 1;
    HS_REQUIRE(o.newton_steps >= -1 && o.newton_steps <= 8, E_PARAM, "Newton steps must be in -1..8");
    HS_REQUIRE(o.mask_mode == 0 || o.mask_mode == 1, E_PARAM, "mask mode must be 0 or 1");
    const bool avg = o.mask_mode == 1;
    // normalize-and-t-th-power (t = 2: normalize-and-square)
    const int tp = o.power > 0 ? o.power : 2;
    HS_REQUIRE(tp >= 2 && tp <= 4, E_PARAM, "power must be 2, 3 or 4");
    HS_REQUIRE(o.approx == 0 || o.approx == 1, E_PARAM, "approx must be 0 (minimax) or 1 (interpolation)");
    HS_REQUIRE(tp == 2 || !smb, E_PARAM, "version B normalizes with squares (power 2)");
    HS_REQUIRE(o.newton_steps <= 0 || tp == 2, E_PARAM,
               "Newton's iteration computes inverse square roots: normalisation with squares");
    // Newton's steps on every inverse square root (Algorithm SM; version B:
    // its last step, the only one that takes an inverse square root): as
    // asked; by default none up to n = 2048 and, above, two (where a
    // degree-255 polynomial alone leaves a relative error near 2^-5 on
    // [~1/n, 1]; each step squares it)
    const int nsteps_opt = o.newton_steps > 0 ? o.newton_steps
                           : (o.newton_steps == 0 && tp == 2 && n > 2048 ? 2 : 0);
    const int tl = tp == 2 ? 1 : 2;         // levels of y^tp
    const int L = (int)((long long)m * N0 / np2);
    // Theorem "th:prec_softmax"'s k (M / t^k ~ ln n for the t-th power
    // variant); from n = 4096 one more iteration, which narrows the first
    // normalisation interval [e^(-t M / t^k), 1]
    const int k = o.k > 0 ? o.k : power_k(n, M, tp) + (n >= 4096 ? 1 : 0);
    const int per = np2 / m;
    const int nrot = ilog2(per);
    // the jobs' auxiliary ciphertexts packed into one (version B with
    // squares and the indicator mask, no Newton steps, J L <= N/2)
    HS_REQUIRE(o.merge == 0 || (smb && !avg && nsteps_opt == 0 && (J <= per || J % per == 0)), E_PARAM,
               "Softmax: packed auxiliary ciphertexts for several jobs need version B, the indicator mask, no "
               "Newton steps and jobs <= n / m or a multiple of it");
    const bool mg = o.merge != 0 && J > 1;
    const int Jg = std::min(J, per);          // jobs per packed auxiliary ciphertext
    const double Delta = std::ldexp(1.0, c.prm.log_scale);
    // rotation keys for the rotate-and-add loops (strides +-L 2^t)
    for (int t = 0; t < nrot; t++) {
        add_galois_key(c, galois_rot(-(L << t), c.N));
        add_galois_key(c, galois_rot(L << t, c.N));
    }
    // v = 2x / M in [-2, 0]: a change of the declared scale when the input
    // was encrypted at scale ~ 2 Delta / M; one rescale first when it was
    // encrypted at (2 Delta / M) q_l (its encryption noise, about 2^17 of
    // the scale's unit in the slots at N = 2^16, then shrinks by q_l: at
    // scale 2 Delta / M itself that noise, about 2^-16.6 in logit units, is
    // the largest error of the output, since Softmax passes an absolute
    // logit error on as a relative output error); otherwise one constant
    // product.
    Ct v;
    const double vs = x.scale * M / 2.0;
    if (std::fabs(std::log2(vs) - c.prm.log_scale) <= 2.0) {
        v = ct_copy(c, x);
        v.scale = vs;
    } else if (x.level >= 1 && std::fabs(std::log2(vs / (double)c.primes[x.level]) - c.prm.log_scale) <= 2.0) {
        v = op_rescale(c, x);
        v.scale = v.scale * M / 2.0;
    } else {
        v = op_mul_const(c, x, 2.0 / M, Delta);
    }
    // y0 = exp(x / t^k) / n^(1/t)  (the prescale keeps sum y0^t in
    // [e^(-t M / t^k), 1])
    const double isn = tp == 2 ? 1.0 / std::sqrt((double)n) : std::pow((double)n, -1.0 / tp);
    const quad Mq = M;
    const int kk = k;
    const quad tk2 = tp == 2 ? ldexpq(1, kk + 1) : 2 * powq((quad)tp, (quad)kk);
    ChebPoly pexp = cheb_fit([&](quad u) { return expq(Mq * u / tk2) * (quad)isn; }, -2.0, 0.0, o.exp_degree);
    Ct y0 = eval_cheb(c, v, pexp, Delta);
    ct_free(c, v);
    if (np2 != n) {
        Ct ym = mask_padding(c, y0, n, per, L, m);
        ct_free(c, y0);
        y0 = ym;
    }
    if (o.debug_stop == 0) return y0;
    // the factor's slots: [0, L), or [0, J L) on the packed ciphertext
    const double* mask = mask_coeffs(c, mg ? Jg * L : L);

    Ct y = ct_copy(c, y0);      // y^(j-1)
    Ct big;                     // Lambda (version B), on slots [0, L) only
    bool have_big = false;
    double ybound = isn * 1.05; // bound on |y^(j-1)| for its bootstrapping
    double lo = (tp == 2 ? std::exp(-2.0 * M / std::ldexp(1.0, k)) : std::exp(-tp * M / std::pow((double)tp, k))) * 0.98;
    double hi = 1.0;
    for (int j = 1; j <= k; j++) {
        const bool last = j == k;
        const bool smb_step = smb && !last;
        const int nsteps = smb_step ? 0 : nsteps_opt;
        // exponent of the normalisation: 1/t (SM, and the last step of B) or 2^-j
        const double e = smb_step ? std::ldexp(1.0, -j) : (tp == 2 ? 0.5 : 1.0 / tp);
        int deg = j == 1 ? o.inv_degree_first : (last ? o.inv_degree_last : o.inv_degree_mid);
        if (deg <= 0) {
            // the paper's depths at n = 256 (6, 5, 7) for n <= 256 (its table
            // has depth 4 in the middle at n = 128; 5 is kept here, on the
            // power-of-two-wide intervals); above, one more level for the
            // first and middle steps (the relative error at the low end of
            // [~1/n, 1] would otherwise widen every later interval)
            // t-th powers: the later intervals [~n^-(t-1), 1] are far wider,
            // so depth 6 / 7 up to n = 16 and 7 above
            int d;
            if (tp != 2) d = n <= 16 ? (last ? 7 : 6) : 7;
            else if (n <= 256) d = j == 1 ? 6 : (last ? 7 : 5);
            else if (n <= 1024) d = last ? 8 : 6;
            else d = last ? 8 : 7;
            deg = (1 << d) - 1;
        }
        // main thread: this iteration's z = lambda y and z^t (1 + tl levels),
        // then the levels of the next y^t feeding S
        if (!smb) {
            bool rep;
            Ct y2 = ensure_level(c, y, last ? 1 + tl : 1 + 2 * tl, ybound, st, rep, "y", j);
            if (rep) {
                ct_free(c, y);
                y = y2;
            }
        }
        // auxiliary thread, powering: S = sum over the m ciphertexts of y^t
        // (squares: one relinearisation for the whole sum)
        Ct S;
        if (tp == 2) {
            Ct d = op_square_sum_jobs(c, y, J);
            Ct r = op_relin(c, d);
            ct_free(c, d);
            S = op_rescale(c, r);
            ct_free(c, r);
        } else {
            Ct yt = op_power(c, y, tp);
            S = op_sum_jobs(c, yt, J);
            ct_free(c, yt);
        }
        // auxiliary thread, summation: rotate-and-add with strides -L 2^t
        for (int t = 0; t < nrot; t++) {
            Ct rr = op_rotate(c, S, -(L << t));
            op_add_inplace(c, S, rr);
            ct_free(c, rr);
        }
        if (mg) {
            Ct Sp = pack_jobs(c, S, L, Jg);
            ct_free(c, S);
            S = Sp;
        }
        // budget of the normalisation polynomial (mask folded into its leaves,
        // or into the last Newton step): lambda lands cheb_depth (+ 1 when
        // the affine map takes a level) + 2 nsteps below S; the cube and
        // fourth power variants and Newton's steps also keep 1 + tl levels in
        // lambda for z = lambda y and z^t.  When that exceeds the level a
        // bootstrapping restores, Newton's first guess P(S) is bootstrapped
        // itself before the steps (S then needs the polynomial's depth and,
        // one level above the guess, the steps' levels)
        // The last step's z = lambda y and z^2 take two of lambda's levels
        // (earlier steps of Algorithm SM bootstrap lambda when it is short;
        // version B's Lambda product takes one); packed jobs: one more for
        // taking the factor apart before the normalize-and-square step.
        const int keep = ((tp != 2 || nsteps) ? 2 + tl : (last ? 1 + tl : 1)) + (mg && !smb_step ? 1 : 0);
        const int need_full = cheb_depth(deg) + 2 * nsteps + keep;
        const bool refresh = nsteps > 0 && can_bootstrap(c) && need_full > c.prm.user_top;
        {
            const int needS = refresh ? std::max(cheb_depth(deg), 2 * nsteps + keep + 1) : need_full;
            bool rep;
            Ct S2 = ensure_level(c, S, needS, hi * 1.1, st, rep, "S", j);
            if (rep) {
                ct_free(c, S);
                S = S2;
            }
        }
        // the interval of the normalisation polynomial: [lo, lo + 2^w], whose
        // affine map is an integer product; in the last iteration of Algorithm
        // SM with squares (the polynomial whose error reaches the output),
        // exactly [lo, hi] when S has the level its affine map then takes on
        // top of the polynomial and the final z = lambda y, y = z^2 (about 4
        // bits of precision at n = 256: the wider interval spends the
        // approximation on values S never takes)
        double a, b;
        if (last && tp == 2 && !nsteps && S.level >= cheb_depth(deg) + 3 + (mg ? 1 : 0)) {
            a = lo;
            b = hi;
        } else {
            free_interval(lo, hi, a, b);
        }
        // the paper's weighted minimax approximant (smallest max |P(s) s^e - 1|),
        // or the Chebyshev interpolant
        const quad eq = e;
        ChebPoly pinv = o.approx == 0 ? minimax_invpow(a, b, deg, e)
                                      : cheb_fit([&](quad s) { return powq(s, -eq); }, a, b, deg);
        const double delta0 = rel_error(pinv, lo, hi, e);
        const double delta = newton_delta(delta0, nsteps);
        double lam_bound = (nsteps ? (1.0 + delta) / std::sqrt(lo) : max_abs(pinv, lo, hi)) * 1.05;
        // the averaging mask: per copies of the factor, each divided by per,
        // summed by the broadcast (the division folded into the coefficients
        // when there is no Newton step, exact since per is a power of two)
        ChebPoly pe = pinv;
        if (avg && !nsteps)
            for (double& cf : pe.c) cf /= per;
        if (avg) lam_bound /= per;
        // normalisation and mask: lambda = P(S) * mask, on slots [0, L)
        // (averaging: P(S) / per on every slot)
        Ct lam;
        if (!nsteps) {
            lam = eval_cheb(c, S, pe, Delta, avg ? nullptr : mask);
        } else {
            Ct g = eval_cheb(c, S, pinv, Delta);
            if (refresh) {
                bool rep;
                Ct g2 = ensure_level(c, g, 2 * nsteps + keep, (1.0 + delta0) / std::sqrt(lo) * 1.05, st, rep,
                                     "guess", j);
                if (rep) {
                    ct_free(c, g);
                    g = g2;
                }
                if (g.level >= S.level) {
                    Ct gd = ct_drop(c, g, S.level - 1);
                    ct_free(c, g);
                    g = gd;
                }
            }
            lam = newton_invsqrt(c, S, g, nsteps, avg ? nullptr : mask, avg ? per : 1, Delta);
            ct_free(c, g);
        }
        ct_free(c, S);
        if (!smb_step) {
            // SM step (and the last step of version B): z = lambda y, y = z^t.
            // y ends at min(y, lambda) - 1 - tl; bootstrap lambda (masked,
            // before its broadcast) only when it is the ciphertext that leaves
            // y short of the next iteration's need (1 + 2 tl, or 1 + tl
            // before the last step).
            const int need_next = (j + 1 == k) ? 1 + tl : 1 + 2 * tl;
            if (!last && can_bootstrap(c) && lam.level < y.level && lam.level - 1 - tl < need_next) {
                bool rep;
                Ct l2 = ensure_level(c, lam, y.level, lam_bound, st, rep, "lambda", j, avg ? 0 : L);
                if (rep) {
                    ct_free(c, lam);
                    lam = l2;
                }
            }
            if (mg) {
                Ct lu = unpack_jobs(c, lam, J, L, Jg);
                ct_free(c, lam);
                lam = lu;
            }
            broadcast(c, lam, L, nrot);
            Ct lj = per_job(c, lam, J, m);
            ct_free(c, lam);
            Ct z = op_mult(c, y, lj);
            ct_free(c, lj);
            ct_free(c, y);
            y = op_power(c, z, tp);
            ct_free(c, z);
            // sum y^(j) in [(1 - delta)^t, (1 + delta)^t], so by the power-mean
            // inequality sum (y^(j))^t in [(1 - delta)^(t^2) / n^(t-1), (1 + delta)^(t^2)]
            if (tp == 2) {
                lo = std::pow(1.0 - delta, 4.0) / n * 0.98;
                hi = std::pow(1.0 + delta, 4.0) * 1.0001;
            } else {
                lo = std::pow(1.0 - delta, (double)(tp * tp)) / std::pow((double)n, tp - 1.0) * 0.98;
                hi = std::pow(1.0 + delta, (double)(tp * tp)) * 1.0001;
            }
            ybound = hi * 1.05;
        } else {
            // version B: Lambda = Lambda * lambda_j (both on slots [0, L));
            // z = broadcast(Lambda) y0; y = z^(2^j).  Averaging mask: lambda_j
            // broadcast first (the average of its copies on every slot), so
            // Lambda is kept on every slot and needs no broadcast
            if (avg) broadcast(c, lam, L, nrot);
            if (!have_big) {
                big = lam;
                have_big = true;
            } else {
                Ct nb = op_mult(c, big, lam);
                ct_free(c, big);
                ct_free(c, lam);
                big = nb;
            }
            // y^(j) = (Lambda y0)^(2^j) must keep r levels: 1 for the next
            // S, 2 before the final normalize-and-square step (packed jobs:
            // 2 always, the next S's packing taking one); packed, Lambda
            // keeps one more for taking the jobs' factors apart
            const int r = (j == k - 1 || mg) ? 2 : 1;
            const int want = j + 1 + r;
            HS_REQUIRE(y0.level >= want, E_LEVEL, "Softmax version B: main-thread level budget exhausted");
            const int want_big = want + (mg ? 1 : 0);
            if (big.level < want_big) {
                bool rep;
                Ct b2 = ensure_level(c, big, want_big, lam_bound_big(n, avg ? lam_bound * per : lam_bound), st,
                                     rep, "Lambda", j, avg ? 0 : (mg ? Jg * L : L));
                if (rep) {
                    ct_free(c, big);
                    big = b2;
                }
            }
            Ct bb = mg ? unpack_jobs(c, big, J, L, Jg) : ct_copy(c, big);
            if (!avg) broadcast(c, bb, L, nrot);
            Ct bj = per_job(c, bb, J, m);
            ct_free(c, bb);
            Ct z = op_mult(c, y0, bj);
            ct_free(c, bj);
            ct_free(c, y);
            y = z;
            for (int s = 0; s < j; s++) {
                Ct y2 = op_mult(c, y, y);
                ct_free(c, y);
                y = y2;
            }
            const double ej = std::ldexp(1.0, j + 1);
            lo = std::pow(1.0 - delta, ej) / n * 0.98;
            hi = std::pow(1.0 + delta, ej) * 1.0001;
        }
        st.levels_left = y.level;
        if (o.debug_stop == j) break;
    }
    ct_free(c, y0);
    if (have_big) ct_free(c, big);
    st.k = k;
    if (stats) *stats = st;
    return y;
}

}  // namespace hs
