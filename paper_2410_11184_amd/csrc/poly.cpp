// Polynomial approximation and homomorphic polynomial evaluation.
//
// The paper evaluates exp and x^(-1/2^j) by polynomial approximations of
// degree 2^t - 1 (Section 5.1, "Designing auxiliary functions"), in
// ceil(log(d+1)) levels and O(sqrt d) products (Section 2.2, "Functions as
// polynomials", Paterson-Stockmeyer).  Here:
//  * coefficients: Chebyshev interpolation at the d+1 first-kind nodes,
//    computed in binary128 and rounded once to double;
//  * evaluation: baby-step giant-step in the Chebyshev basis.  Baby steps
//    T_1..T_{B-1} by T_2k = 2 T_k^2 - 1 and T_2k+1 = 2 T_k T_k+1 - T_1; giant
//    steps T_B, T_2B, ...; the polynomial splits as q_lo + q_hi T_n
//    (T_n+i = 2 T_n T_i - T_n-i).  Every addition is scale-exact: each leaf
//    sum_j c_j T_j multiplies T_j by the integer rint(c_j S q / s_j) so that
//    all terms share the scale S q before the single rescale of the leaf.
//    Depth: ceil(log2(d+1)) + 1 (the +1 is the leaf's constant products).
#include <algorithm>
#include <cmath>
#include <complex>
#include <functional>
#include <map>

#include <quadmath.h>

#include "host.h"
#include "poly.h"

namespace hs {

ChebPoly cheb_fit(const std::function<quad(quad)>& f, double a, double b, int d) {
    ChebPoly p;
    p.a = a;
    p.b = b;
    p.c.assign(d + 1, 0.0);
    std::vector<quad> fx(d + 1);
    const quad pi = M_PIq;
    for (int k = 0; k <= d; k++) {
        const quad u = cosq(pi * (k + (quad)0.5) / (d + 1));
        const quad x = (u * ((quad)b - (quad)a) + (quad)a + (quad)b) / 2;
        fx[k] = f(x);
    }
    for (int j = 0; j <= d; j++) {
        quad s = 0;
        for (int k = 0; k <= d; k++) s += fx[k] * cosq(pi * j * (k + (quad)0.5) / (d + 1));
        quad cj = (quad)2 / (d + 1) * s;
        if (j == 0) cj /= 2;
        p.c[j] = (double)cj;
    }
    return p;
}

double cheb_eval_plain(const ChebPoly& p, double x) {
    const double u = (2 * x - p.a - p.b) / (p.b - p.a);
    double b1 = 0, b2 = 0;
    for (int j = (int)p.c.size() - 1; j >= 1; j--) {
        const double t = 2 * u * b1 - b2 + p.c[j];
        b2 = b1;
        b1 = t;
    }
    return u * b1 - b2 + p.c[0];
}

static int ceil_log2(int x) {
    int l = 0;
    while ((1 << l) < x) l++;
    return l;
}

int cheb_depth(int degree) { return ceil_log2(degree + 1) + 1; }

// ---------------------------------------------------------------- evaluator
u64* mask_plaintext(Context& c, const double* mask, int lv, double scale, bool* owned) {
    const auto key = std::make_tuple(mask, lv, scale);
    auto it = c.mask_pts.find(key);
    *owned = false;
    if (it != c.mask_pts.end()) return it->second;
    const size_t bytes = sizeof(u64) * (size_t)(lv + 1) * c.N;
    const bool keep = c.mask_pts_bytes + bytes <= Context::kMaskCacheBytes;
    u64* pt = keep ? (u64*)c.persistent_alloc(bytes, "mask plaintext") : c.alloc_words((size_t)(lv + 1) * c.N);
    Rows r = c.rows(pt, 1, lv + 1, (size_t)(lv + 1) * c.N);
    k_encode_real(c.T, r, mask, 0, scale, c.stream);
    k_ntt(c.T, r, false, c.stream);
    if (keep) {
        c.mask_pts[key] = pt;
        c.mask_pts_bytes += bytes;
    } else {
        *owned = true;
    }
    return pt;
}

namespace {

using cplx = std::complex<double>;

struct Val {
    bool is_const = false;
    cplx cval = 0;
    Ct ct;
};

struct Evaluator {
    Context& c;
    std::map<int, Ct> T;          // Chebyshev basis polynomials of u
    std::map<std::pair<int, double>, Ct> t1_at;  // T_1 adjusted to (level, exact scale)
    int B = 2;
    // When set: every leaf constant c is replaced by the plaintext c * mask
    // (mask = device coefficients of a 0/1 slot vector), which multiplies the
    // whole polynomial by the mask since mask^2 = mask.
    const double* mask = nullptr;

    u64* mask_pt(double scale, int lv, bool* owned) { return mask_plaintext(c, mask, lv, scale, owned); }

    // a (level lv) * (value * mask) with the product at scale a.scale * pscale
    Ct mul_mask(const Ct& a, double value, double pscale) {
        bool owned;
        u64* pt = mask_pt(value * pscale, a.level, &owned);
        Ct o = op_mul_plain(c, a, pt, pscale, false);
        if (owned) c.free_words(pt);
        return o;
    }

    void add_mask_const(Ct& a, double value) {
        bool owned;
        u64* pt = mask_pt(value * a.scale, a.level, &owned);
        Rows r0 = c.comp_rows(a, 0);
        Rows rp{pt, a.m, a.level + 1, 0, a.level + 1, 0, c.nq};
        c.count(OC_ADD, a.level, a.m / 2.0);
        k_add(c.T, r0, r0, rp, c.stream);
        if (owned) c.free_words(pt);
    }

    explicit Evaluator(Context& cc) : c(cc) {}
    ~Evaluator() {
        for (auto& kv : T) ct_free(c, kv.second);
        for (auto& kv : t1_at) ct_free(c, kv.second);
    }

    // T_1 brought to (level, scale) by a scale-exact constant product
    const Ct& t1_adjusted(int level, double scale) {
        // keyed by the exact scale: scales of one level differ by the primes'
        // offsets from a power of two (~2^-40 relative), and a T_1 at a
        // neighbouring scale would add that relative error to T_j
        auto k = std::make_pair(level, scale);
        auto it = t1_at.find(k);
        if (it != t1_at.end()) return it->second;
        const Ct& t1 = T.at(1);
        HS_REQUIRE(t1.level > level, E_LEVEL, "polynomial evaluation: level budget exhausted");
        Ct d = ct_drop(c, t1, level + 1);
        Ct r = op_mul_const(c, d, 1.0, scale);
        ct_free(c, d);
        return t1_at.emplace(k, r).first->second;
    }

    Ct mult_aligned(const Ct& a, const Ct& b) { return op_mult(c, a, b); }

    void build_T(int j) {
        if (T.count(j)) return;
        if (j % 2 == 0) {
            build_T(j / 2);
            Ct s = mult_aligned(T.at(j / 2), T.at(j / 2));
            op_mul_int_inplace(c, s, 2);
            op_add_const_inplace(c, s, -1.0);
            T[j] = s;
        } else {
            build_T((j + 1) / 2);
            build_T((j - 1) / 2);
            Ct s = mult_aligned(T.at((j + 1) / 2), T.at((j - 1) / 2));
            op_mul_int_inplace(c, s, 2);
            const Ct& t1 = t1_adjusted(s.level, s.scale);
            op_sub_inplace(c, s, t1);
            T[j] = s;
        }
    }

    static void accumulate(Context& c, Ct& acc, bool& have, Ct& t) {
        if (!have) {
            acc = t;
            have = true;
        } else {
            op_add_inplace(c, acc, t);
            ct_free(c, t);
        }
    }

    // sum_j coef[j] T_j at (scale S, level lv); one rescale.  Every term
    // T_j (read at level lv + 1) times its integer round(coef S q / scale_j),
    // or times its masked plaintext, enters one multiply-accumulate launch;
    // imaginary parts are summed apart and multiplied by X^(N/2), which
    // multiplies every slot by i exactly (no level, no noise).
    Val leaf(const std::vector<cplx>& coef, double S, int lv) {
        int deg = (int)coef.size() - 1;
        while (deg > 0 && coef[deg] == 0.0) deg--;
        Val v;
        if (deg == 0) {
            v.is_const = true;
            v.cval = coef.empty() ? 0.0 : coef[0];
            return v;
        }
        const double ql = (double)c.primes[lv + 1];
        std::vector<LeafTerm> terms[2];
        std::vector<u64*> owned_pts;   // uncached mask plaintexts, freed after the launches
        int m = 0;
        for (int j = 1; j <= deg; j++) {
            if (coef[j] == 0.0) continue;
            build_T(j);
            const Ct& tj = T.at(j);
            HS_REQUIRE(tj.level >= lv + 1, E_LEVEL, "polynomial evaluation: level budget exhausted");
            m = tj.m;
            for (int part = 0; part < 2; part++) {
                const double value = part == 0 ? coef[j].real() : coef[j].imag();
                if (value == 0.0) continue;
                LeafTerm t{};
                t.a = tj.d;
                t.arows = tj.level + 1;
                if (mask) {
                    HS_REQUIRE(part == 0, E_ARG, "masked evaluation takes real coefficients");
                    bool owned;
                    const double pscale = S * ql / tj.scale;
                    u64* pt = mask_pt(value * pscale, lv + 1, &owned);
                    if (owned) owned_pts.push_back(pt);
                    t.p = pt;
                } else {
                    const double K = std::rint(value * S * ql / tj.scale);
                    if (K == 0.0) continue;   // the term vanishes at this scale
                    const double a = std::fabs(K);
                    t.neg = K < 0;
                    if (a < 9.2e18) {
                        t.mant = (u64)a;
                        t.e = 0;
                    } else {
                        int e;
                        const double mant = std::frexp(a, &e);
                        t.mant = (u64)std::ldexp(mant, 53);
                        t.e = e - 53;
                    }
                }
                terms[part].push_back(t);
            }
        }
        Ct acc;
        bool have = false;
        for (int part = 0; part < 2; part++) {
            if (terms[part].empty()) continue;
            Ct s = ct_alloc(c, m, 2, lv + 1);
            s.scale = S * ql;
            c.count(OC_PTMUL, lv + 1, (double)m * terms[part].size());
            c.count(OC_ADD, lv + 1, (double)m * (terms[part].size() - 1));
            k_leaf_mac(c.T, s.d, 2 * m, lv + 2, terms[part].data(), (int)terms[part].size(), c.stream);
            if (part == 1) {
                Ct t = op_mul_monomial(c, s, c.N / 2);
                ct_free(c, s);
                s = t;
            }
            accumulate(c, acc, have, s);
        }
        for (u64* pt : owned_pts) c.free_words(pt);
        if (!have) {
            // every term rounded to zero
            acc = ct_alloc(c, std::max(m, 1), 2, lv + 1);
            acc.scale = S * ql;
            k_zero_rows(c.T, c.ct_rows(acc), c.stream);
        }
        HS_REQUIRE(coef[0].imag() == 0.0, E_ARG, "polynomial evaluation: imaginary constant term");
        if (mask) add_mask_const(acc, coef[0].real());
        else op_add_const_inplace(c, acc, coef[0].real());
        v.ct = op_rescale(c, acc);
        ct_free(c, acc);
        v.ct.scale = S;
        return v;
    }

    // g * cv at scale S (one rescale): real and imaginary parts apart
    Ct mul_const_complex(const Ct& g, cplx cv, double S) {
        Ct r;
        bool have = false;
        if (cv.real() != 0.0) {
            Ct t = op_mul_const(c, g, cv.real(), S);
            accumulate(c, r, have, t);
        }
        if (cv.imag() != 0.0) {
            Ct t = op_mul_const(c, g, cv.imag(), S);
            Ct ti = op_mul_monomial(c, t, c.N / 2);
            ct_free(c, t);
            accumulate(c, r, have, ti);
        }
        HS_REQUIRE(have, E_ARG, "polynomial evaluation: zero leading part");
        return r;
    }

    Val eval(const std::vector<cplx>& coef, double S, int lv) {
        int deg = (int)coef.size() - 1;
        while (deg > 0 && coef[deg] == 0.0) deg--;
        if (deg < B) return leaf(std::vector<cplx>(coef.begin(), coef.begin() + deg + 1), S, lv);
        int n = B;
        while (2 * n <= deg) n *= 2;
        // p = q_lo + q_hi T_n
        std::vector<cplx> hi(deg - n + 1), lo(n);
        hi[0] = coef[n];
        for (int k = 1; k <= deg - n; k++) hi[k] = 2.0 * coef[n + k];
        for (int j = 0; j < n; j++) lo[j] = coef[j];
        for (int k = 1; k <= deg - n; k++) lo[n - k] -= coef[n + k];
        build_T(n);
        const Ct& G = T.at(n);
        HS_REQUIRE(G.level >= lv + 1, E_LEVEL, "polynomial evaluation: level budget exhausted");
        const double ql = (double)c.primes[lv + 1];
        Val vh = eval(hi, S * ql / G.scale, lv + 1);
        Val out;
        Ct g = ct_drop(c, G, lv + 1);
        if (vh.is_const && mask) {
            HS_REQUIRE(vh.cval.imag() == 0.0, E_ARG, "masked evaluation takes real coefficients");
            Ct t = mul_mask(g, vh.cval.real(), S * ql / g.scale);
            out.ct = op_rescale(c, t);
            ct_free(c, t);
            out.ct.scale = S;
        } else if (vh.is_const) {
            out.ct = mul_const_complex(g, vh.cval, S);
        } else {
            Ct d = op_tensor(c, vh.ct, g);
            Ct r = op_relin(c, d);
            ct_free(c, d);
            out.ct = op_rescale(c, r);
            ct_free(c, r);
            ct_free(c, vh.ct);
            out.ct.scale = S;
        }
        ct_free(c, g);
        Val vl = eval(lo, S, lv);
        if (vl.is_const) {
            HS_REQUIRE(vl.cval.imag() == 0.0, E_ARG, "polynomial evaluation: imaginary constant term");
            if (mask) add_mask_const(out.ct, vl.cval.real());
            else op_add_const_inplace(c, out.ct, vl.cval.real());
        } else {
            op_add_inplace(c, out.ct, vl.ct);
            ct_free(c, vl.ct);
        }
        return out;
    }
};

}  // namespace

Ct eval_cheb_complex(Context& c, const Ct& x, const ChebPoly& re, const ChebPoly& im, double target_scale) {
    HS_REQUIRE(re.a == -1.0 && re.b == 1.0 && im.a == -1.0 && im.b == 1.0, E_ARG,
               "complex evaluation expects polynomials on [-1, 1]");
    const size_t n = std::max(re.c.size(), im.c.size());
    std::vector<cplx> coef(n, 0.0);
    for (size_t j = 0; j < n; j++)
        coef[j] = cplx(j < re.c.size() ? re.c[j] : 0.0, j < im.c.size() ? im.c[j] : 0.0);
    const int d = (int)n - 1;
    HS_REQUIRE(d >= 1, E_ARG, "polynomial degree must be >= 1");
    const int t = ceil_log2(d + 1);
    const int out_level = x.level - (t + 1);
    HS_REQUIRE(out_level >= 0, E_LEVEL, "polynomial evaluation: level budget exhausted");
    Evaluator ev(c);
    ev.B = 1 << std::max(1, (t + 1) / 2);
    ev.T[1] = ct_copy(c, x);
    Val v = ev.eval(coef, target_scale, out_level);
    HS_REQUIRE(!v.is_const, E_ARG, "constant polynomial");
    return v.ct;
}

Ct eval_cheb(Context& c, const Ct& x, const ChebPoly& p, double target_scale, const double* mask) {
    const int d = (int)p.c.size() - 1;
    HS_REQUIRE(d >= 1, E_ARG, "polynomial degree must be >= 1");
    // affine map to u in [-1, 1]: u = alpha x + beta
    const double alpha = 2.0 / (p.b - p.a);
    const double beta = -(p.a + p.b) / (p.b - p.a);
    Ct u;
    int ea = 0;
    const double fa = std::frexp(alpha, &ea);  // alpha = fa 2^ea, fa in [0.5, 1)
    if (fa == 0.5 && ea >= 1) {
        // alpha = 2^(ea-1) >= 1: integer product, no level used
        u = ct_copy(c, x);
        op_mul_int_inplace(c, u, 1LL << (ea - 1));
    } else {
        HS_REQUIRE(x.level >= 1, E_LEVEL, "polynomial evaluation: level budget exhausted");
        u = op_mul_const(c, x, alpha, std::ldexp(1.0, c.prm.log_scale));
    }
    op_add_const_inplace(c, u, beta);
    const int t = ceil_log2(d + 1);
    const int out_level = u.level - (t + 1);
    HS_REQUIRE(out_level >= 0, E_LEVEL, "polynomial evaluation: level budget exhausted");
    Evaluator ev(c);
    ev.mask = mask;
    ev.B = 1 << std::max(1, (t + 1) / 2);
    ev.T[1] = u;
    Val v = ev.eval(std::vector<cplx>(p.c.begin(), p.c.end()), target_scale, out_level);
    HS_REQUIRE(!v.is_const, E_ARG, "constant polynomial");
    return v.ct;
}

}  // namespace hs
