// Chebyshev approximations and their homomorphic evaluation.
#pragma once
#include <functional>
#include <vector>

#include "host.h"

namespace hs {

// p(x) = sum_j c[j] T_j((2x - a - b) / (b - a)) on [a, b]
struct ChebPoly {
    double a = -1, b = 1;
    std::vector<double> c;
};

// Interpolation at the degree + 1 Chebyshev nodes of the first kind, every
// step in binary128 (f too), so the coefficients are the exact interpolant's
// rounded to the nearest double: the same doubles any correct high-precision
// computation of that interpolant gives.
typedef __float128 quad;
ChebPoly cheb_fit(const std::function<quad(quad)>& f, double a, double b, int degree);
// The weighted minimax approximant of s^-e on [a, b] (Section 5.1,
// "Designing auxiliary functions": P minimising max |P(s) s^e - 1|), degree
// d, in the Chebyshev basis of [a, b], as the discrete minimax on the grid
// u_i = -cos(pi i / (G - 1)), i < G = 16 (d + 1) + 1, by the Remez exchange:
// reference = grid indices 16 k (the extrema of T_(d+1)), k = 0..d+1; each
// round (at most 40, 80-bit arithmetic) solves the reference system
// sum_j c_j T_j(u_k) + (-1)^k h / w_k = 1 / w_k (w = s^e), takes in every
// run of equal sign of r = w P - 1 on the grid the index of the largest |r|
// (the first on ties), drops end candidates (the one with the smaller |r|,
// the last on ties) down to d + 2, and stops when fewer remain, the
// reference repeats, or the levelled error |h| of the round's system is
// below 2^-40 (then before the exchange); the coefficients are those of the
// final reference
// system solved in binary128, each rounded to the nearest multiple of
// 2^(E - 52), 2^E <= max_j |c_j| < 2^(E+1).  Cached per (a, b, d, e).
ChebPoly minimax_invpow(double a, double b, int d, double e);
double cheb_eval_plain(const ChebPoly& p, double x);
int cheb_depth(int degree);   // levels used by eval_cheb (plus 1 if the affine map needs one)
// Evaluate p on every slot of the batch x; result at scale target_scale.
// With `mask` (device array of the N real coefficients of a 0/1 slot vector,
// laid out as encode_to lays out w), the result is p(x) * mask at no extra
// level: every leaf constant becomes a masked plaintext.
Ct eval_cheb(Context& c, const Ct& x, const ChebPoly& p, double target_scale, const double* mask = nullptr);
// NTT-domain rows 0..lv of rint(scale * w), w = `mask` (device coefficients of
// a slot vector, laid out as encode_to lays them out): from the context's
// cache (built on first use and kept, *owned = false), else in a pool buffer
// the caller frees (*owned = true)
u64* mask_plaintext(Context& c, const double* mask, int lv, double scale, bool* owned);
// re(x) + i im(x) for two polynomials on [-1, 1], as one polynomial with
// complex coefficients (the imaginary parts through a product by X^(N/2),
// which multiplies every slot by i): half the products of evaluating both.
// Every constant term met must be real (HS_E_ARG otherwise).
Ct eval_cheb_complex(Context& c, const Ct& x, const ChebPoly& re, const ChebPoly& im, double target_scale);

}  // namespace hs
