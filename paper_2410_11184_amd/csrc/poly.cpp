// Polynomial approximation and homomorphic polynomial evaluation.
//
// The paper evaluates exp and x^(-1/2^j) by polynomial approximations of
// degree 2^t - 1 (Section 5.1, "Designing auxiliary functions"), in
// ceil(log(d+1)) levels and O(sqrt d) products (Section 2.2, "Functions as
// polynomials", Paterson-Stockmeyer).  Here:
//  * coefficients: Chebyshev interpolation at the d+1 first-kind nodes,
//    computed in binary128 and rounded once to double (the exponential); for
//    the inverse powers s^-e, the paper's weighted minimax approximants
//    (minimal max |P(s) s^e - 1|) by a Remez exchange on a fixed grid;
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
#include <mutex>
#include <tuple>

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

// ------------------------------------------------ weighted minimax (Remez)
namespace {

typedef long double ld;

// Solve A x = y (n x n, row-major, destroyed) by Gaussian elimination with
// partial pivoting.
template <class T>
std::vector<T> gauss_solve(std::vector<T>& A, std::vector<T> y, int n, T (*fab)(T)) {
    for (int col = 0; col < n; col++) {
        int piv = col;
        for (int r = col + 1; r < n; r++)
            if (fab(A[(size_t)r * n + col]) > fab(A[(size_t)piv * n + col])) piv = r;
        HS_REQUIRE(A[(size_t)piv * n + col] != 0, E_ARG, "minimax: singular reference system");
        if (piv != col) {
            for (int j = 0; j < n; j++) std::swap(A[(size_t)piv * n + j], A[(size_t)col * n + j]);
            std::swap(y[piv], y[col]);
        }
        const T inv = 1 / A[(size_t)col * n + col];
        for (int r = col + 1; r < n; r++) {
            const T f = A[(size_t)r * n + col] * inv;
            if (f == 0) continue;
            for (int j = col; j < n; j++) A[(size_t)r * n + j] -= f * A[(size_t)col * n + j];
            y[r] -= f * y[col];
        }
    }
    std::vector<T> x(n);
    for (int r = n - 1; r >= 0; r--) {
        T s = y[r];
        for (int j = r + 1; j < n; j++) s -= A[(size_t)r * n + j] * x[j];
        x[r] = s / A[(size_t)r * n + r];
    }
    return x;
}

ld fabs_ld(ld v) { return v < 0 ? -v : v; }
quad fabs_q(quad v) { return v < 0 ? -v : v; }

// The reference system at grid indices ref: sum_j c_j T_j(u_k) + (-1)^k h / w_k
// = 1 / w_k, w = s^e; returns c_0..c_d, h.
template <class T>
std::vector<T> reference_solve(const std::vector<int>& ref, int d, int G, double a, double b, T e, T pi,
                               T (*cosfn)(T), T (*powfn)(T, T), T (*fab)(T)) {
    const int n = d + 2;
    std::vector<T> A((size_t)n * n), y(n);
    for (int k = 0; k < n; k++) {
        const T u = -cosfn(pi * (T)ref[k] / (T)(G - 1));
        const T s = (u * ((T)b - (T)a) + (T)a + (T)b) / 2;
        const T w = powfn(s, e);
        T t0 = 1, t1 = u;
        A[(size_t)k * n] = 1;
        if (d >= 1) A[(size_t)k * n + 1] = u;
        for (int j = 2; j <= d; j++) {
            const T t2 = 2 * u * t1 - t0;
            A[(size_t)k * n + j] = t2;
            t0 = t1;
            t1 = t2;
        }
        A[(size_t)k * n + d + 1] = ((k & 1) ? -1 : 1) / w;
        y[k] = 1 / w;
    }
    return gauss_solve<T>(A, y, n, fab);
}

ld cos_ld(ld v) { return cosl(v); }
ld pow_ld(ld v, ld e) { return powl(v, e); }
quad cos_q(quad v) { return cosq(v); }
quad pow_q(quad v, quad e) { return powq(v, e); }

}  // namespace

ChebPoly minimax_invpow(double a, double b, int d, double e) {
    static std::mutex mu;
    static std::map<std::tuple<double, double, int, double>, ChebPoly> cache;
    HS_REQUIRE(d >= 0 && d <= 1023 && a > 0 && b > a && e > 0, E_ARG, "minimax: bad interval, degree or power");
    const auto key = std::make_tuple(a, b, d, e);
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
    }
    const int G = 16 * (d + 1) + 1;
    const ld pi = 3.141592653589793238462643383279502884L;
    // grid, weights, and T_j on the grid (80-bit)
    std::vector<ld> u(G), w(G);
    for (int i = 0; i < G; i++) {
        u[i] = -cosl(pi * (ld)i / (ld)(G - 1));
        const ld s = (u[i] * ((ld)b - (ld)a) + (ld)a + (ld)b) / 2;
        w[i] = powl(s, (ld)e);
    }
    std::vector<int> ref(d + 2);
    for (int k = 0; k <= d + 1; k++) ref[k] = 16 * k;
    std::vector<ld> r(G);
    for (int it = 0; it < 40; it++) {
        const std::vector<ld> c = reference_solve<ld>(ref, d, G, a, b, (ld)e, pi, cos_ld, pow_ld, fabs_ld);
        // levelled error below 2^-40: far below any ciphertext's precision,
        // and near the 80-bit rounding of r, where the exchange would follow
        // rounding noise
        if (fabs_ld(c[d + 1]) < 0x1p-40L) break;
        for (int i = 0; i < G; i++) {
            // Clenshaw
            ld b1 = 0, b2 = 0;
            for (int j = d; j >= 1; j--) {
                const ld t = 2 * u[i] * b1 - b2 + c[j];
                b2 = b1;
                b1 = t;
            }
            r[i] = w[i] * (u[i] * b1 - b2 + c[0]) - 1;
        }
        // one candidate per run of equal sign: its largest |r| (first on ties)
        std::vector<int> cand;
        int start = 0;
        for (int i = 1; i <= G; i++) {
            if (i == G || (r[i] >= 0) != (r[start] >= 0)) {
                int best = start;
                for (int q = start + 1; q < i; q++)
                    if (fabs_ld(r[q]) > fabs_ld(r[best])) best = q;
                cand.push_back(best);
                start = i;
            }
        }
        // too many: drop the end candidate with the smaller |r| (the last on ties)
        while ((int)cand.size() > d + 2) {
            if (fabs_ld(r[cand.front()]) < fabs_ld(r[cand.back()])) cand.erase(cand.begin());
            else cand.pop_back();
        }
        if ((int)cand.size() < d + 2 || cand == ref) break;
        ref = cand;
    }
    // final solve at the reference in binary128
    const std::vector<quad> cq = reference_solve<quad>(ref, d, G, a, b, (quad)e, M_PIq, cos_q, pow_q, fabs_q);
    // every coefficient to the nearest multiple of the largest one's double
    // ulp 2^(E - 52), 2^E <= max |c_j| < 2^(E+1): coefficients far below the
    // largest are then as reproducible as the largest (the high-order ones of
    // a near-exact fit are otherwise at the solve's rounding level)
    quad cmax = 0;
    for (int j = 0; j <= d; j++) cmax = std::max(cmax, fabs_q(cq[j]));
    int E = 0;
    frexpq(cmax, &E);   // cmax = f 2^E, f in [0.5, 1)
    const int sh = (E - 1) - 52;
    ChebPoly p;
    p.a = a;
    p.b = b;
    p.c.resize(d + 1);
    for (int j = 0; j <= d; j++) p.c[j] = (double)(rintq(ldexpq(cq[j], -sh)) * ldexpq(1, sh));
    std::lock_guard<std::mutex> g(mu);
    cache[key] = p;
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
