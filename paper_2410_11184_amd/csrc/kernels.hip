// HIP kernels for RNS-CKKS ring arithmetic on CDNA4 (gfx950).
//
// Every polynomial is a set of rows ("limbs") of N 64-bit residues, one row
// per prime, in the negacyclic NTT domain unless a kernel says otherwise.
// Arithmetic is on the VALU: 64-bit products from 32-bit multiplies, Shoup
// multiplication by precomputed constants (twiddles, conversion constants)
// and Barrett reduction for products of two variables.  All kernels keep
// values fully reduced in [0, q) at their boundaries.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "dev.h"

namespace hs {

// ------------------------------------------------------------- profiler
struct Profiler {
    bool on = false;
    struct Rec {
        int kind;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> spare;
    hipEvent_t get() {
        if (!spare.empty()) {
            hipEvent_t e = spare.back();
            spare.pop_back();
            return e;
        }
        hipEvent_t e;
        (void)hipEventCreate(&e);
        return e;
    }
};

Profiler* prof_create() { return new Profiler(); }
void prof_destroy(Profiler* p) {
    if (!p) return;
    for (auto& r : p->recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : p->spare) (void)hipEventDestroy(e);
    delete p;
}
void prof_enable(Profiler* p, bool on) {
    if (p) p->on = on;
}
bool prof_enabled(const Profiler* p) { return p && p->on; }
void prof_collect(Profiler* p, double* out) {
    for (int k = 0; k < 3 * PK_COUNT; k++) out[k] = 0;
    if (!p) return;
    for (auto& r : p->recs) {
        (void)hipEventSynchronize(r.b);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, r.a, r.b);
        out[3 * r.kind] += 1;
        out[3 * r.kind + 1] += ms;
        out[3 * r.kind + 2] += r.bytes;
        p->spare.push_back(r.a);
        p->spare.push_back(r.b);
    }
    p->recs.clear();
}

// RAII scope recording an event pair around the launches it encloses
struct ProfScope {
    Profiler* p;
    hipStream_t st;
    hipEvent_t a{}, b{};
    int kind;
    double bytes;
    ProfScope(Profiler* pp, int k, double by, void* stream) : p(pp), st((hipStream_t)stream), kind(k), bytes(by) {
        if (p && p->on) {
            a = p->get();
            (void)hipEventRecord(a, st);
        }
    }
    ~ProfScope() {
        if (p && p->on) {
            b = p->get();
            (void)hipEventRecord(b, st);
            p->recs.push_back({kind, a, b, bytes});
        }
    }
};

// autotuner decisions (defined with the tuner below)
int tune_ntt16(const DevTables& T, const Rows& x, bool inverse, hipStream_t st, const NttSkip* skip = nullptr);
int tune_conv(const DevTables& T, const ConvTables& C, size_t og, size_t ig, int ngroups, hipStream_t st);

// ------------------------------------------------------------- arithmetic
__device__ __forceinline__ u64 add_mod(u64 a, u64 b, u64 q) {
    u64 s = a + b;
    return s >= q ? s - q : s;
}
__device__ __forceinline__ u64 sub_mod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + q - b; }

// a * w mod q for any a < 2^64, w < q, ws = floor(w 2^64 / q)
__device__ __forceinline__ u64 mul_shoup(u64 a, u64 w, u64 ws, u64 q) {
    u64 hi = __umul64hi(a, ws);
    u64 r = a * w - hi * q;
    return r >= q ? r - q : r;
}

// Barrett reduction of the 128-bit x = (hi, lo) < 2^(2b) (HAC 14.42, base 2)
__device__ __forceinline__ u64 barrett128(u64 hi, u64 lo, const PrimeInfo& P) {
    const int b = P.bits;
    u64 x1 = (hi << (65 - b)) | (lo >> (b - 1));
    u64 plo = x1 * P.mu;
    u64 phi = __umul64hi(x1, P.mu);
    u64 qh = (phi << (63 - b)) | (plo >> (b + 1));
    u64 r = lo - qh * P.q;
    if (r >= P.q) r -= P.q;
    if (r >= P.q) r -= P.q;
    return r;
}

__device__ __forceinline__ u64 mul_mod(u64 a, u64 b, const PrimeInfo& P) {
    return barrett128(__umul64hi(a, b), a * b, P);
}

// x mod q for any 64-bit x (valid since 2^64 <= 2^(2b) for b >= 32)
__device__ __forceinline__ u64 reduce64(u64 x, const PrimeInfo& P) { return barrett128(0, x, P); }

// w mod q for w < 2^128 given r64 = 2^64 mod q: (hi mod q) r64 + lo mod q
__device__ __forceinline__ u64 reduce_wide(unsigned __int128 w, const PrimeInfo& P, u64 r64) {
    const u64 h = reduce64((u64)(w >> 64), P);
    return add_mod(mul_mod(h, r64, P), reduce64((u64)w, P), P.q);
}

__device__ __forceinline__ int prime_of(const Rows& x, int r) {
    return r < x.nq ? x.q_off + r : x.p_base + (r - x.nq);
}

__device__ __forceinline__ u64* row_ptr(const Rows& x, int row, int N) {
    int g = row / x.rpg;
    int r = row - g * x.rpg;
    return x.base + (size_t)g * x.gstride + (size_t)r * N;
}

// ------------------------------------------------------------ Philox4x32-10
__device__ __forceinline__ void philox(u64 seed, u64 domain, u64 index, u32 out[4]) {
    u32 c0 = (u32)index, c1 = (u32)(index >> 32), c2 = (u32)domain, c3 = (u32)(domain >> 32);
    u32 k0 = (u32)seed, k1 = (u32)(seed >> 32);
#pragma unroll
    for (int r = 0; r < 10; r++) {
        u64 p0 = (u64)0xD2511F53u * c0;
        u64 p1 = (u64)0xCD9E8D57u * c2;
        u32 n0 = (u32)(p1 >> 32) ^ c1 ^ k0;
        u32 n1 = (u32)p1;
        u32 n2 = (u32)(p0 >> 32) ^ c3 ^ k1;
        u32 n3 = (u32)p0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// ------------------------------------------------------------------ NTT
// Forward: Cooley-Tukey with psi^brv twiddles, natural order in, bit-reversed
// evaluation order out.  Inverse: Gentleman-Sande with psi^-brv, then N^-1.
// N <= 4096: one workgroup holds a whole row in LDS.  Larger N: N = R * C;
// pass 1 runs the first log R stages on LDS tiles of R rows x TC columns
// (stride-C elements), pass 2 the last log C stages on TR contiguous chunks
// of C elements.

__global__ void __launch_bounds__(256) ntt_small_kernel(DevTables T, Rows x, int inverse) {
    extern __shared__ u64 sm[];
    const int N = T.N, logN = T.logN;
    const int row = blockIdx.x;
    u64* p = row_ptr(x, row, N);
    const int pi = prime_of(x, row % x.rpg);
    const u64 q = T.prime[pi].q;
    for (int e = threadIdx.x; e < N; e += blockDim.x) sm[e] = p[e];
    __syncthreads();
    const int half = N >> 1;
    if (!inverse) {
        const u64* w = T.tw + (size_t)pi * N;
        const u64* ws = T.tws + (size_t)pi * N;
        for (int s = 0; s < logN; s++) {
            const int m = 1 << s;
            const int lt = logN - 1 - s;  // log t
            for (int k = threadIdx.x; k < half; k += blockDim.x) {
                const int i = k >> lt;
                const int j = k & ((1 << lt) - 1);
                const int j1 = (i << (lt + 1)) + j;
                const u64 W = w[m + i], Ws = ws[m + i];
                const u64 u = sm[j1];
                const u64 v = mul_shoup(sm[j1 + (1 << lt)], W, Ws, q);
                sm[j1] = add_mod(u, v, q);
                sm[j1 + (1 << lt)] = sub_mod(u, v, q);
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < N; e += blockDim.x) p[e] = sm[e];
    } else {
        const u64* w = T.itw + (size_t)pi * N;
        const u64* ws = T.itws + (size_t)pi * N;
        for (int s = logN - 1; s >= 0; s--) {
            const int m = 1 << s;
            const int lt = logN - 1 - s;
            for (int k = threadIdx.x; k < half; k += blockDim.x) {
                const int i = k >> lt;
                const int j = k & ((1 << lt) - 1);
                const int j1 = (i << (lt + 1)) + j;
                const u64 W = w[m + i], Ws = ws[m + i];
                const u64 u = sm[j1];
                const u64 v = sm[j1 + (1 << lt)];
                sm[j1] = add_mod(u, v, q);
                sm[j1 + (1 << lt)] = mul_shoup(sub_mod(u, v, q), W, Ws, q);
            }
            __syncthreads();
        }
        const u64 ni = T.ninv[2 * pi], nis = T.ninv[2 * pi + 1];
        for (int e = threadIdx.x; e < N; e += blockDim.x) p[e] = mul_shoup(sm[e], ni, nis, q);
    }
}

// pass 1: stages m = 1 .. R/2 (forward) or R/2 .. 1 (inverse, then * N^-1)
__global__ void __launch_bounds__(256) ntt_pass1_kernel(DevTables T, Rows x, int logR, int logC,
                                                        int logTC, int inverse) {
    extern __shared__ u64 sm[];
    const int N = T.N;
    const int R = 1 << logR, C = 1 << logC, TC = 1 << logTC;
    const int row = blockIdx.y;
    const int c0 = blockIdx.x * TC;
    u64* p = row_ptr(x, row, N);
    const int pi = prime_of(x, row % x.rpg);
    const u64 q = T.prime[pi].q;
    for (int e = threadIdx.x; e < R * TC; e += blockDim.x) {
        const int rr = e >> logTC, cc = e & (TC - 1);
        sm[e] = p[(size_t)rr * C + c0 + cc];
    }
    __syncthreads();
    const int nb = (R >> 1) * TC;
    if (!inverse) {
        const u64* w = T.tw + (size_t)pi * N;
        const u64* ws = T.tws + (size_t)pi * N;
        for (int s = 0; s < logR; s++) {
            const int m = 1 << s;
            const int ltr = logR - 1 - s;
            for (int k = threadIdx.x; k < nb; k += blockDim.x) {
                const int cc = k & (TC - 1);
                const int kk = k >> logTC;
                const int i = kk >> ltr;
                const int jr = kk & ((1 << ltr) - 1);
                const int r0 = (i << (ltr + 1)) + jr;
                const int a0 = (r0 << logTC) + cc, a1 = ((r0 + (1 << ltr)) << logTC) + cc;
                const u64 u = sm[a0];
                const u64 v = mul_shoup(sm[a1], w[m + i], ws[m + i], q);
                sm[a0] = add_mod(u, v, q);
                sm[a1] = sub_mod(u, v, q);
            }
            __syncthreads();
        }
        for (int e = threadIdx.x; e < R * TC; e += blockDim.x) {
            const int rr = e >> logTC, cc = e & (TC - 1);
            p[(size_t)rr * C + c0 + cc] = sm[e];
        }
    } else {
        const u64* w = T.itw + (size_t)pi * N;
        const u64* ws = T.itws + (size_t)pi * N;
        for (int s = logR - 1; s >= 0; s--) {
            const int m = 1 << s;
            const int ltr = logR - 1 - s;
            for (int k = threadIdx.x; k < nb; k += blockDim.x) {
                const int cc = k & (TC - 1);
                const int kk = k >> logTC;
                const int i = kk >> ltr;
                const int jr = kk & ((1 << ltr) - 1);
                const int r0 = (i << (ltr + 1)) + jr;
                const int a0 = (r0 << logTC) + cc, a1 = ((r0 + (1 << ltr)) << logTC) + cc;
                const u64 u = sm[a0];
                const u64 v = sm[a1];
                sm[a0] = add_mod(u, v, q);
                sm[a1] = mul_shoup(sub_mod(u, v, q), w[m + i], ws[m + i], q);
            }
            __syncthreads();
        }
        const u64 ni = T.ninv[2 * pi], nis = T.ninv[2 * pi + 1];
        for (int e = threadIdx.x; e < R * TC; e += blockDim.x) {
            const int rr = e >> logTC, cc = e & (TC - 1);
            p[(size_t)rr * C + c0 + cc] = mul_shoup(sm[e], ni, nis, q);
        }
    }
}

// pass 2: stages m = R .. N/2 (forward) or N/2 .. R (inverse)
__global__ void __launch_bounds__(256) ntt_pass2_kernel(DevTables T, Rows x, int logR, int logC,
                                                        int logTR, int inverse) {
    extern __shared__ u64 sm[];
    const int N = T.N;
    const int R = 1 << logR, C = 1 << logC, TR = 1 << logTR;
    const int row = blockIdx.y;
    const int rc0 = blockIdx.x * TR;
    u64* p = row_ptr(x, row, N) + (size_t)rc0 * C;
    const int pi = prime_of(x, row % x.rpg);
    const u64 q = T.prime[pi].q;
    for (int e = threadIdx.x; e < TR * C; e += blockDim.x) sm[e] = p[e];
    __syncthreads();
    const int nb = TR * (C >> 1);
    const u64* w = (inverse ? T.itw : T.tw) + (size_t)pi * N;
    const u64* ws = (inverse ? T.itws : T.tws) + (size_t)pi * N;
    for (int step = 0; step < logC; step++) {
        const int s = inverse ? (logC - 1 - step) : step;
        const int m = R << s;
        const int lt = logC - 1 - s;  // log t
        for (int k = threadIdx.x; k < nb; k += blockDim.x) {
            const int rr = k >> (logC - 1);
            const int kk = k & ((C >> 1) - 1);
            const int gi = kk >> lt;
            const int j = kk & ((1 << lt) - 1);
            const int e0 = (rr << logC) + (gi << (lt + 1)) + j;
            const int e1 = e0 + (1 << lt);
            const int i = ((rc0 + rr) << (logC - 1 - lt)) + gi;
            const u64 W = w[m + i], Ws = ws[m + i];
            const u64 u = sm[e0];
            if (!inverse) {
                const u64 v = mul_shoup(sm[e1], W, Ws, q);
                sm[e0] = add_mod(u, v, q);
                sm[e1] = sub_mod(u, v, q);
            } else {
                const u64 v = sm[e1];
                sm[e0] = add_mod(u, v, q);
                sm[e1] = mul_shoup(sub_mod(u, v, q), W, Ws, q);
            }
        }
        __syncthreads();
    }
    for (int e = threadIdx.x; e < TR * C; e += blockDim.x) p[e] = sm[e];
}

// ---- N = 2^16: two passes of 256-point sub-transforms (index j = 16 hi + lo)
// on tiles of 16 sub-transforms.  Pass 1 takes stages 0..7 on columns
// (stride 256), pass 2 stages 8..15 on contiguous chunks of 256.  Each thread
// keeps 16 elements in registers and runs 4 stages on them (radix 16); one
// LDS exchange switches from the hi-stages to the lo-stages.  The twiddle of
// stage s, group i is tw[2^s + i]; on 16 registers spanning local bits 3..0
// with prefix P it is tw[((2^S0 + P) << a) + g] for local stage a, group g.
// Rows are visited prime-major so that the twiddles of one prime stay in L2.
// Both passes belong to one transform (k_ntt): the rows between them hold
// values in [0, 4q) (forward) or [0, 2q) (inverse).

__device__ __forceinline__ int ntt_row_prime_major(const Rows& x, int y) {
    const int g = y % x.ngroups;
    return g * x.rpg + y / x.ngroups;
}

// row visited by workgroup row y: prime-major (order 0) or in storage order
// (1); with a skip, y enumerates only the transformed rows (vrows per group,
// rows of groups with fewer get -1) and g0 is the launch's first group
__device__ __forceinline__ int ntt_row(const Rows& x, int y, int order, const NttSkip& sk, int g0) {
    if (!sk.per) return order ? y : ntt_row_prime_major(x, y);
    const int own_min = sk.nql - ((sk.nql - 1) / sk.digit) * sk.digit;
    const int V = x.rpg - own_min;
    const int g = order ? y / V : y % x.ngroups;
    const int rv = order ? y % V : y / x.ngroups;
    const int lo = ((g0 + g) % sk.per) * sk.digit;
    const int own = min(lo + sk.digit, sk.nql) - lo;
    const int r = rv < lo ? rv : rv + own;
    return r < x.rpg ? g * x.rpg + r : -1;
}

// Lazy (Harvey) butterflies: a*w - floor(a*ws/2^64)*q lies in [0, 2q) for
// any a < 2^64, so forward values are kept in [0, 4q) and inverse values in
// [0, 2q) (4q < 2^63 for q < 2^61) and reduced once at the end of the
// transform; between the two passes the rows hold these unreduced values.
__device__ __forceinline__ u64 mul_shoup_lazy(u64 a, u64 w, u64 ws, u64 nq) {
    return a * w + __umul64hi(a, ws) * nq;
}

__device__ __forceinline__ void fwd16(u64 (&E)[16], const ulonglong2* tw, u32 base, u64 q, u64 nq) {
    ulonglong2 W[15];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int g = 0; g < (1 << a); g++) W[(1 << a) - 1 + g] = tw[(base << a) + g];
    const u64 q2 = 2 * q;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const int h = 8 >> a;
#pragma unroll
        for (int g = 0; g < (1 << a); g++) {
            const ulonglong2 w = W[(1 << a) - 1 + g];
#pragma unroll
            for (int j = 0; j < h; j++) {
                const int k = g * 2 * h + j;
                u64 u = E[k];
                u = u >= q2 ? u - q2 : u;
                const u64 v = mul_shoup_lazy(E[k + h], w.x, w.y, nq);
                E[k] = u + v;
                E[k + h] = u - v + q2;
            }
        }
    }
}

__device__ __forceinline__ void inv16(u64 (&E)[16], const ulonglong2* tw, u32 base, u64 q, u64 nq) {
    ulonglong2 W[15];
#pragma unroll
    for (int a = 0; a < 4; a++)
#pragma unroll
        for (int g = 0; g < (1 << a); g++) W[(1 << a) - 1 + g] = tw[(base << a) + g];
    const u64 q2 = 2 * q;
#pragma unroll
    for (int a = 3; a >= 0; a--) {
        const int h = 8 >> a;
#pragma unroll
        for (int g = 0; g < (1 << a); g++) {
            const ulonglong2 w = W[(1 << a) - 1 + g];
#pragma unroll
            for (int j = 0; j < h; j++) {
                const int k = g * 2 * h + j;
                const u64 u = E[k], v = E[k + h];
                const u64 s = u + v;
                E[k] = s >= q2 ? s - q2 : s;
                E[k + h] = mul_shoup_lazy(u - v + q2, w.x, w.y, nq);
            }
        }
    }
}

// [0, 4q) -> [0, q)
__device__ __forceinline__ u64 reduce4q(u64 x, u64 q) {
    x = x >= 2 * q ? x - 2 * q : x;
    return x >= q ? x - q : x;
}

// Tiles of C columns (pass 1) or C chunks of 256 (pass 2) per workgroup of
// 16 C threads, C = 16 or 8 (a tuner choice: 8 doubles the workgroups of a
// launch); every element sees the same butterflies either way.  LDS layouts
// (u64 units), conflict-free for both access patterns of each pass:
// pass 1 element (hi, lo, column c) at hi*17C + lo*C + c,
// pass 2 element (chunk w, hi, lo) at w*272 + hi*17 + lo.

// centred lift of x (mod q_s) to the prime of P: x if x <= (q_s - 1) / 2,
// else x - q_s, reduced
__device__ __forceinline__ u64 lift_centred(u64 x, u64 qs, const PrimeInfo& P) {
    if (x <= (qs - 1) / 2) return reduce64(x, P);
    const u64 mag = reduce64(qs - x, P);
    return mag ? P.q - mag : 0;
}

template <int C>
__global__ void __launch_bounds__(16 * C) ntt16_p1_kernel(DevTables T, Rows x, Rows src, int inverse, int order,
                                                         NttSkip sk, int g0, NttLift lf) {
    constexpr int S1 = 17 * C;
    __shared__ u64 sm[16 * S1];
    const int row = ntt_row(x, blockIdx.y, order, sk, g0);
    if (row < 0) return;   // whole workgroup
    u64* p = row_ptr(x, row, 65536) + blockIdx.x * C;
    const u64* ps = row_ptr(src, row, 65536) + blockIdx.x * C;
    const int pi = prime_of(x, row % x.rpg);
    const u64 q = T.prime[pi].q;
    const u64 nq = T.prime[pi].nq;
    const int t = threadIdx.x, c = t % C, hl = t / C;
    u64 E[16];
    if (!inverse) {
        const ulonglong2* tw = (const ulonglong2*)T.tw2 + (size_t)pi * 65536;
        // thread (lo = hl, c): hi = 0..15, stages 0..3
        if (lf.base) {
            const PrimeInfo P = T.prime[pi];
            const u64 qs = T.prime[lf.src_prime].q;
            const u64* pl = lf.base + (size_t)(row / x.rpg) * lf.gs + blockIdx.x * C;
#pragma unroll
            for (int hi = 0; hi < 16; hi++) E[hi] = lift_centred(pl[(size_t)(hi * 16 + hl) * 256 + c], qs, P);
        } else {
#pragma unroll
            for (int hi = 0; hi < 16; hi++) E[hi] = ps[(size_t)(hi * 16 + hl) * 256 + c];
        }
        fwd16(E, tw, 1, q, nq);
#pragma unroll
        for (int hi = 0; hi < 16; hi++) sm[hi * S1 + hl * C + c] = E[hi];
        __syncthreads();
        // thread (hi = hl, c): lo = 0..15, stages 4..7
#pragma unroll
        for (int lo = 0; lo < 16; lo++) E[lo] = sm[hl * S1 + lo * C + c];
        fwd16(E, tw, 16 + hl, q, nq);
#pragma unroll
        for (int lo = 0; lo < 16; lo++) p[(size_t)(hl * 16 + lo) * 256 + c] = E[lo];
    } else {
        const ulonglong2* tw = (const ulonglong2*)T.itw2 + (size_t)pi * 65536;
        // thread (hi = hl, c): lo = 0..15, stages 7..4
#pragma unroll
        for (int lo = 0; lo < 16; lo++) E[lo] = ps[(size_t)(hl * 16 + lo) * 256 + c];
        inv16(E, tw, 16 + hl, q, nq);
#pragma unroll
        for (int lo = 0; lo < 16; lo++) sm[hl * S1 + lo * C + c] = E[lo];
        __syncthreads();
        // thread (lo = hl, c): hi = 0..15, stages 3..0, then N^-1
#pragma unroll
        for (int hi = 0; hi < 16; hi++) E[hi] = sm[hi * S1 + hl * C + c];
        inv16(E, tw, 1, q, nq);
        const u64 ni = T.ninv[2 * pi], nis = T.ninv[2 * pi + 1];
#pragma unroll
        for (int hi = 0; hi < 16; hi++) p[(size_t)(hi * 16 + hl) * 256 + c] = mul_shoup(E[hi], ni, nis, q);
    }
}

// four waves per SIMD: the LDS tile (35 KB per 256-thread workgroup) allows
// four workgroups per CU, and 128 VGPRs (no spills) lets the registers follow
template <bool EPI, int C>
__global__ void __launch_bounds__(16 * C) __attribute__((amdgpu_waves_per_eu(4, 8))) ntt16_p2_kernel(DevTables T, Rows x, Rows src, int inverse, int order,
                                                       NttEpilogue Ep, NttSkip sk) {
    __shared__ u64 sm[C * 272];
    const int row = ntt_row(x, blockIdx.y, order, sk, Ep.g0);
    if (row < 0) return;   // whole workgroup
    const int pi = prime_of(x, row % x.rpg);
    const u64 q = T.prime[pi].q;
    const u64 nq = T.prime[pi].nq;
    const int t = threadIdx.x, w = t >> 4, l = t & 15;
    const u32 R = blockIdx.x * C + w;              // chunk index
    u64* p = row_ptr(x, row, 65536) + (size_t)R * 256;
    const u64* ps = row_ptr(src, row, 65536) + (size_t)R * 256;
    const ulonglong2* tw = (const ulonglong2*)(inverse ? T.itw2 : T.tw2) + (size_t)pi * 65536;
    u64* s = sm + w * 272;
    u64 E[16];
    // coalesced load: thread (w, lo = l) takes hi = 0..15
#pragma unroll
    for (int hi = 0; hi < 16; hi++) E[hi] = ps[hi * 16 + l];
    if (!inverse) {
        fwd16(E, tw, 256 + R, q, nq);                   // stages 8..11
#pragma unroll
        for (int hi = 0; hi < 16; hi++) s[hi * 17 + l] = E[hi];
        __syncthreads();
        // thread (w, hi = l): lo = 0..15, stages 12..15 (in place in LDS)
#pragma unroll
        for (int lo = 0; lo < 16; lo++) E[lo] = s[l * 17 + lo];
        fwd16(E, tw, 4096 + R * 16 + l, q, nq);
#pragma unroll
        for (int lo = 0; lo < 16; lo++) s[l * 17 + lo] = E[lo];
        __syncthreads();
        if constexpr (!EPI) {
#pragma unroll
            for (int hi = 0; hi < 16; hi++) p[hi * 16 + l] = reduce4q(s[hi * 17 + l], q);
        } else {
            // (d +) (a - NTT(x)) c for this row, written to its destination
            const int G = Ep.g0 + row / x.rpg, r = row % x.rpg;
            const int j = G % Ep.split, gj = G / Ep.split;
            const size_t off = (size_t)r * 65536 + (size_t)R * 256;
            const u64* pa = Ep.a + (size_t)G * Ep.a_gs + off;
            u64* po = Ep.out[j] + (size_t)gj * Ep.out_gs[j] + off;
            const u64 c = Ep.c.c[r], cs = Ep.c.cs[r];
#pragma unroll
            for (int hi = 0; hi < 16; hi++) {
                const int k = hi * 16 + l;
                u64 v = sub_mod(pa[k], reduce4q(s[hi * 17 + l], q), q);
                if (Ep.mul) v = mul_shoup(v, c, cs, q);
                if (Ep.d[j]) v = add_mod(Ep.d[j][(size_t)gj * Ep.d_gs[j] + off + k], v, q);
                po[k] = v;
            }
        }
    } else {
#pragma unroll
        for (int hi = 0; hi < 16; hi++) s[hi * 17 + l] = E[hi];
        __syncthreads();
        // thread (w, hi = l): lo = 0..15, stages 15..12
#pragma unroll
        for (int lo = 0; lo < 16; lo++) E[lo] = s[l * 17 + lo];
        inv16(E, tw, 4096 + R * 16 + l, q, nq);
#pragma unroll
        for (int lo = 0; lo < 16; lo++) s[l * 17 + lo] = E[lo];
        __syncthreads();
        // thread (w, lo = l): hi = 0..15, stages 11..8
#pragma unroll
        for (int hi = 0; hi < 16; hi++) E[hi] = s[hi * 17 + l];
        inv16(E, tw, 256 + R, q, nq);
#pragma unroll
        for (int hi = 0; hi < 16; hi++) p[hi * 16 + l] = E[hi];
    }
}

void k_ntt(const DevTables& T, const Rows& x, bool inverse, void* stream) { k_ntt_from(T, x, x, inverse, stream); }

// N = 2^16 transform of x (first pass reading src) in one of the tuner's
// variants: variant & 1 selects the row order (prime-major / storage order),
// variant & 2 splits the launch into batches of kNttGroupBatch row groups,
// variant & 4 takes tiles of 8 columns / chunks (128-thread workgroups, twice
// as many) instead of 16.
constexpr int kNttGroupBatch = 8;
static const char* const kNttVariants[] = {"prime-major",        "storage-order",
                                           "prime-major/batched", "storage-order/batched",
                                           "prime-major/tile8",   "storage-order/tile8",
                                           "prime-major/batched/tile8", "storage-order/batched/tile8"};
static void ntt16_launch(const DevTables& T, const Rows& x, const Rows& src, bool inverse, int variant,
                         hipStream_t st, const NttEpilogue* epi = nullptr, const NttSkip& sk = NttSkip(),
                         const NttLift* lift = nullptr) {
    const int order = variant & 1;
    const int gb = (variant & 2) ? kNttGroupBatch : x.ngroups;
    const int vrows = sk.per ? x.rpg - (sk.nql - ((sk.nql - 1) / sk.digit) * sk.digit) : x.rpg;
    NttEpilogue e;
    if (epi) e = *epi;
    for (int g0 = 0; g0 < x.ngroups; g0 += gb) {
        Rows xs = x, ss = src;
        xs.base = x.base + (size_t)g0 * x.gstride;
        ss.base = src.base + (size_t)g0 * src.gstride;
        xs.ngroups = ss.ngroups = std::min(gb, x.ngroups - g0);
        e.g0 = g0;
        NttLift lf;
        if (lift) {
            lf = *lift;
            lf.base = lift->base + (size_t)g0 * lift->gs;
        }
        const int rows = xs.ngroups * vrows;
        if (!(variant & 4)) {
            const dim3 g(16, rows);
            if (!inverse) {
                hipLaunchKernelGGL(ntt16_p1_kernel<16>, g, dim3(256), 0, st, T, xs, ss, 0, order, sk, g0, lf);
                if (epi)
                    hipLaunchKernelGGL((ntt16_p2_kernel<true, 16>), g, dim3(256), 0, st, T, xs, xs, 0, order, e, sk);
                else
                    hipLaunchKernelGGL((ntt16_p2_kernel<false, 16>), g, dim3(256), 0, st, T, xs, xs, 0, order, e, sk);
            } else {
                hipLaunchKernelGGL((ntt16_p2_kernel<false, 16>), g, dim3(256), 0, st, T, xs, ss, 1, order, e, sk);
                hipLaunchKernelGGL(ntt16_p1_kernel<16>, g, dim3(256), 0, st, T, xs, xs, 1, order, sk, g0, NttLift());
            }
        } else {
            const dim3 g(32, rows);
            if (!inverse) {
                hipLaunchKernelGGL(ntt16_p1_kernel<8>, g, dim3(128), 0, st, T, xs, ss, 0, order, sk, g0, lf);
                if (epi)
                    hipLaunchKernelGGL((ntt16_p2_kernel<true, 8>), g, dim3(128), 0, st, T, xs, xs, 0, order, e, sk);
                else
                    hipLaunchKernelGGL((ntt16_p2_kernel<false, 8>), g, dim3(128), 0, st, T, xs, xs, 0, order, e, sk);
            } else {
                hipLaunchKernelGGL((ntt16_p2_kernel<false, 8>), g, dim3(128), 0, st, T, xs, ss, 1, order, e, sk);
                hipLaunchKernelGGL(ntt16_p1_kernel<8>, g, dim3(128), 0, st, T, xs, xs, 1, order, sk, g0, NttLift());
            }
        }
    }
}

void k_ntt_skip(const DevTables& T, const Rows& x, const NttSkip& skip, void* stream) {
    if (x.ngroups * x.rpg == 0) return;
    if (T.logN != 16 || !skip.per) {
        k_ntt(T, x, false, stream);
        return;
    }
    hipStream_t st = (hipStream_t)stream;
    const int variant = tune_ntt16(T, x, false, st, &skip);
    const int rows = x.ngroups * x.rpg - (x.ngroups / skip.per) * skip.nql;   // transformed rows
    ProfScope ps(T.prof, PK_NTT, 16.0 * T.N * rows, stream);
    ntt16_launch(T, x, x, false, variant, st, nullptr, skip);
}

void k_ntt_epilogue(const DevTables& T, const Rows& x, const NttEpilogue& e, void* stream, const NttLift* lift) {
    const int nrows = x.ngroups * x.rpg;
    if (nrows == 0) return;
    hipStream_t st = (hipStream_t)stream;
    if (T.logN == 16) {
        const int variant = tune_ntt16(T, x, false, st);
        ProfScope ps(T.prof, PK_NTT, 16.0 * T.N * nrows, stream);
        ntt16_launch(T, x, x, false, variant, st, &e, NttSkip(), lift);
        return;
    }
    // other ring sizes: the lift, the transform, then the epilogue as their own kernels
    if (lift) k_lift_centered(T, x, lift->base, lift->gs, lift->src_prime, stream);
    k_ntt(T, x, false, stream);
    for (int j = 0; j < e.split; j++) {
        const int ng = (x.ngroups - j + e.split - 1) / e.split;
        Rows ro{e.out[j], ng, x.rpg, e.out_gs[j], x.nq, x.q_off, x.p_base};
        Rows ra{const_cast<u64*>(e.a) + (size_t)j * e.a_gs, ng, x.rpg, e.a_gs * e.split, x.nq, x.q_off, x.p_base};
        Rows rb{x.base + (size_t)j * x.gstride, ng, x.rpg, x.gstride * e.split, x.nq, x.q_off, x.p_base};
        Rows rd{const_cast<u64*>(e.d[j]), ng, x.rpg, e.d_gs[j], x.nq, x.q_off, x.p_base};
        if (e.mul) {
            if (e.d[j]) k_add_sub_mul_const(T, ro, rd, ra, rb, e.c, stream);
            else k_sub_mul_const(T, ro, ra, rb, e.c, stream);
        } else {
            k_sub(T, ro, ra, rb, stream);
            if (e.d[j]) k_add(T, ro, rd, ro, stream);
        }
    }
}

void k_ntt_from(const DevTables& T, const Rows& x, const Rows& src, bool inverse, void* stream) {
    const int nrows = x.ngroups * x.rpg;
    if (nrows == 0) return;
    hipStream_t st = (hipStream_t)stream;
    if (T.logN == 16) {
        const int variant = tune_ntt16(T, x, inverse, st);
        ProfScope ps(T.prof, PK_NTT, 16.0 * T.N * nrows, stream);
        ntt16_launch(T, x, src, inverse, variant, st);
        return;
    }
    ProfScope ps(T.prof, PK_NTT, 16.0 * T.N * nrows, stream);
    if (src.base != x.base || src.gstride != x.gstride) k_copy_rows(T, x, src, stream);
    if (T.N <= 4096) {
        hipLaunchKernelGGL(ntt_small_kernel, dim3(nrows), dim3(256), T.N * sizeof(u64), st, T, x,
                           inverse ? 1 : 0);
        return;
    }
    const int logC = (T.logN + 1) / 2, logR = T.logN - logC;
    const int logTC = 4, logTR = logR >= 4 ? 4 : logR;
    const dim3 g1((1 << logC) >> logTC, nrows), g2((1 << logR) >> logTR, nrows);
    const size_t lds1 = ((size_t)1 << (logR + logTC)) * sizeof(u64);
    const size_t lds2 = ((size_t)1 << (logC + logTR)) * sizeof(u64);
    if (!inverse) {
        hipLaunchKernelGGL(ntt_pass1_kernel, g1, dim3(256), lds1, st, T, x, logR, logC, logTC, 0);
        hipLaunchKernelGGL(ntt_pass2_kernel, g2, dim3(256), lds2, st, T, x, logR, logC, logTR, 0);
    } else {
        hipLaunchKernelGGL(ntt_pass2_kernel, g2, dim3(256), lds2, st, T, x, logR, logC, logTR, 1);
        hipLaunchKernelGGL(ntt_pass1_kernel, g1, dim3(256), lds1, st, T, x, logR, logC, logTC, 1);
    }
}

// ----------------------------------------------------------- elementwise
// grid: (N / 256, rows); one coefficient per thread
#define EW_INDEX                                  \
    const int row = blockIdx.y;                   \
    const int i = blockIdx.x * blockDim.x + threadIdx.x; \
    const int N = T.N;                            \
    if (i >= N) return;                           \
    const int r = row % out.rpg;                  \
    const PrimeInfo P = T.prime[prime_of(out, r)];

__global__ void add_kernel(DevTables T, Rows out, Rows a, Rows b) {
    EW_INDEX
    row_ptr(out, row, N)[i] = add_mod(row_ptr(a, row, N)[i], row_ptr(b, row, N)[i], P.q);
}
__global__ void sub_kernel(DevTables T, Rows out, Rows a, Rows b) {
    EW_INDEX
    row_ptr(out, row, N)[i] = sub_mod(row_ptr(a, row, N)[i], row_ptr(b, row, N)[i], P.q);
}
__global__ void neg_kernel(DevTables T, Rows out, Rows a) {
    EW_INDEX
    const u64 v = row_ptr(a, row, N)[i];
    row_ptr(out, row, N)[i] = v ? P.q - v : 0;
}
__global__ void mul_kernel(DevTables T, Rows out, Rows a, Rows b) {
    EW_INDEX
    row_ptr(out, row, N)[i] = mul_mod(row_ptr(a, row, N)[i], row_ptr(b, row, N)[i], P);
}
__global__ void mul_add_kernel(DevTables T, Rows out, Rows a, Rows b) {
    EW_INDEX
    u64* o = row_ptr(out, row, N) + i;
    *o = add_mod(*o, mul_mod(row_ptr(a, row, N)[i], row_ptr(b, row, N)[i], P), P.q);
}
__global__ void mul_row_const_kernel(DevTables T, Rows out, Rows a, RowConsts c) {
    EW_INDEX
    row_ptr(out, row, N)[i] = mul_shoup(row_ptr(a, row, N)[i], c.c[r], c.cs[r], P.q);
}
__global__ void add_row_const_kernel(DevTables T, Rows out, Rows a, RowConsts c) {
    EW_INDEX
    row_ptr(out, row, N)[i] = add_mod(row_ptr(a, row, N)[i], c.c[r], P.q);
}
__global__ void sub_mul_const_kernel(DevTables T, Rows out, Rows a, Rows b, RowConsts c) {
    EW_INDEX
    const u64 d = sub_mod(row_ptr(a, row, N)[i], row_ptr(b, row, N)[i], P.q);
    row_ptr(out, row, N)[i] = mul_shoup(d, c.c[r], c.cs[r], P.q);
}
__global__ void add_sub_mul_const_kernel(DevTables T, Rows out, Rows d, Rows a, Rows b, RowConsts c) {
    EW_INDEX
    const u64 t = sub_mod(row_ptr(a, row, N)[i], row_ptr(b, row, N)[i], P.q);
    row_ptr(out, row, N)[i] = add_mod(row_ptr(d, row, N)[i], mul_shoup(t, c.c[r], c.cs[r], P.q), P.q);
}

static inline dim3 ew_grid(const DevTables& T, const Rows& x) {
    return dim3((T.N + 255) / 256, x.ngroups * x.rpg);
}

#define EW_LAUNCH(kern, out, ...)                                                        \
    do {                                                                                 \
        if ((out).ngroups * (out).rpg == 0) return;                                      \
        ProfScope ps_(T.prof, PK_EW, 24.0 * T.N * (out).ngroups * (out).rpg, stream);    \
        hipLaunchKernelGGL(kern, ew_grid(T, out), dim3(256), 0, (hipStream_t)stream, T, out, \
                           __VA_ARGS__);                                                 \
    } while (0)

void k_add(const DevTables& T, const Rows& out, const Rows& a, const Rows& b, void* stream) {
    EW_LAUNCH(add_kernel, out, a, b);
}
void k_sub(const DevTables& T, const Rows& out, const Rows& a, const Rows& b, void* stream) {
    EW_LAUNCH(sub_kernel, out, a, b);
}
void k_neg(const DevTables& T, const Rows& out, const Rows& a, void* stream) { EW_LAUNCH(neg_kernel, out, a); }
// out[R] (+)= sum_t a_t[R] * p_t[R mod rows]: ciphertext rows times
// plaintext rows (broadcast over components and batch), summed mod q.
struct MacTerms {
    const u64* a[kMaxMacTerms];
    const u64* p[kMaxMacTerms];
    int n;
};

__global__ void mul_plain_acc_kernel(DevTables T, u64* out, MacTerms L, int rows, int accumulate) {
    const int R = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = T.N;
    if (i >= N) return;
    const int r = R % rows;
    const PrimeInfo P = T.prime[r];
    const size_t o = (size_t)R * N + i, po = (size_t)r * N + i;
    unsigned __int128 w = accumulate ? out[o] : 0;
    for (int t = 0; t < L.n; t++) w += (unsigned __int128)L.a[t][o] * L.p[t][po];
    out[o] = reduce_wide(w, P, T.r64[r]);
}

void k_mul_plain_acc(const DevTables& T, u64* out, const u64* const* a, const u64* const* p, int nterms,
                     int groups, int rows, void* stream) {
    if (groups * rows == 0 || nterms == 0) return;
    ProfScope ps(T.prof, PK_EW, 8.0 * T.N * groups * rows * (2.0 * nterms + 1), stream);
    for (int t0 = 0; t0 < nterms; t0 += kMaxMacTerms) {
        MacTerms L;
        L.n = std::min(kMaxMacTerms, nterms - t0);
        for (int t = 0; t < L.n; t++) {
            L.a[t] = a[t0 + t];
            L.p[t] = p[t0 + t];
        }
        hipLaunchKernelGGL(mul_plain_acc_kernel, dim3((T.N + 255) / 256, groups * rows), dim3(256), 0,
                           (hipStream_t)stream, T, out, L, rows, t0 > 0 ? 1 : 0);
    }
}

struct LeafTerms {
    LeafTerm t[kMaxMacTerms];
    int n;
};

__global__ void leaf_mac_kernel(DevTables T, u64* out, LeafTerms L, int rows, int accumulate) {
    __shared__ u64 sk[kMaxMacTerms];
    const int R = blockIdx.y;
    const int G = R / rows, r = R - G * rows;
    const PrimeInfo P = T.prime[r];
    // integer constants of the scalar terms, reduced modulo this row's prime
    if (threadIdx.x < L.n && !L.t[threadIdx.x].p) {
        const LeafTerm& lt = L.t[threadIdx.x];
        u64 k = reduce64(lt.mant, P);
        for (int s = 0; s < lt.e; s++) {
            k <<= 1;
            if (k >= P.q) k -= P.q;
        }
        sk[threadIdx.x] = (lt.neg && k) ? P.q - k : k;
    }
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = T.N;
    if (i >= N) return;
    const size_t o = (size_t)R * N + i;
    unsigned __int128 w = accumulate ? out[o] : 0;
    for (int t = 0; t < L.n; t++) {
        const u64 av = L.t[t].a[((size_t)G * L.t[t].arows + r) * N + i];
        const u64 f = L.t[t].p ? L.t[t].p[(size_t)r * N + i] : sk[t];
        w += (unsigned __int128)av * f;
    }
    out[o] = reduce_wide(w, P, T.r64[r]);
}

void k_leaf_mac(const DevTables& T, u64* out, int groups, int rows, const LeafTerm* terms, int nterms,
                void* stream) {
    if (groups * rows == 0 || nterms == 0) return;
    ProfScope ps(T.prof, PK_EW, 8.0 * T.N * groups * rows * (nterms + 1.0), stream);
    for (int t0 = 0; t0 < nterms; t0 += kMaxMacTerms) {
        LeafTerms L;
        L.n = std::min(kMaxMacTerms, nterms - t0);
        for (int t = 0; t < L.n; t++) L.t[t] = terms[t0 + t];
        hipLaunchKernelGGL(leaf_mac_kernel, dim3((T.N + 255) / 256, groups * rows), dim3(256), 0,
                           (hipStream_t)stream, T, out, L, rows, t0 > 0 ? 1 : 0);
    }
}

void k_mul(const DevTables& T, const Rows& out, const Rows& a, const Rows& b, void* stream) {
    EW_LAUNCH(mul_kernel, out, a, b);
}
void k_mul_add(const DevTables& T, const Rows& acc, const Rows& a, const Rows& b, void* stream) {
    EW_LAUNCH(mul_add_kernel, acc, a, b);
}
void k_mul_row_const(const DevTables& T, const Rows& out, const Rows& a, const RowConsts& c, void* stream) {
    EW_LAUNCH(mul_row_const_kernel, out, a, c);
}
void k_add_row_const(const DevTables& T, const Rows& out, const Rows& a, const RowConsts& c, void* stream) {
    EW_LAUNCH(add_row_const_kernel, out, a, c);
}
void k_sub_mul_const(const DevTables& T, const Rows& out, const Rows& a, const Rows& b, const RowConsts& c,
                     void* stream) {
    EW_LAUNCH(sub_mul_const_kernel, out, a, b, c);
}
void k_add_sub_mul_const(const DevTables& T, const Rows& out, const Rows& d, const Rows& a, const Rows& b,
                         const RowConsts& c, void* stream) {
    EW_LAUNCH(add_sub_mul_const_kernel, out, d, a, b, c);
}

// ------------------------------------------------------------- tensor
__global__ void tensor_kernel(DevTables T, Rows d, Rows a, Rows b, size_t ac, size_t bc, size_t dc) {
    const int row = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = T.N;
    if (i >= N) return;
    const int r = row % d.rpg;
    const PrimeInfo P = T.prime[prime_of(d, r)];
    const u64* pa = row_ptr(a, row, N) + i;
    const u64* pb = row_ptr(b, row, N) + i;
    u64* pd = row_ptr(d, row, N) + i;
    const u64 a0 = pa[0], a1 = pa[ac], b0 = pb[0], b1 = pb[bc];
    pd[0] = mul_mod(a0, b0, P);
    pd[dc] = add_mod(mul_mod(a0, b1, P), mul_mod(a1, b0, P), P.q);
    pd[2 * dc] = mul_mod(a1, b1, P);
}

void k_tensor(const DevTables& T, const Rows& d, const Rows& a, const Rows& b, size_t a_comp, size_t b_comp,
              size_t d_comp, void* stream) {
    if (d.ngroups * d.rpg == 0) return;
    ProfScope ps(T.prof, PK_TENSOR, 56.0 * T.N * d.ngroups * d.rpg, stream);
    hipLaunchKernelGGL(tensor_kernel, ew_grid(T, d), dim3(256), 0, (hipStream_t)stream, T, d, a, b, a_comp,
                       b_comp, d_comp);
}

// d = sum over groups g of (a0^2, 2 a0 a1, a1^2)
__global__ void square_sum_kernel(DevTables T, u64* d, size_t dc, Rows a, size_t ac) {
    const int r = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = T.N;
    if (i >= N) return;
    const PrimeInfo P = T.prime[prime_of(a, r)];
    u64 s0 = 0, s1 = 0, s2 = 0;
    for (int g = 0; g < a.ngroups; g++) {
        const u64* pa = a.base + (size_t)g * a.gstride + (size_t)r * N + i;
        const u64 a0 = pa[0], a1 = pa[ac];
        s0 = add_mod(s0, mul_mod(a0, a0, P), P.q);
        const u64 x = mul_mod(a0, a1, P);
        s1 = add_mod(s1, add_mod(x, x, P.q), P.q);
        s2 = add_mod(s2, mul_mod(a1, a1, P), P.q);
    }
    u64* pd = d + (size_t)r * N + i;
    pd[0] = s0;
    pd[dc] = s1;
    pd[2 * dc] = s2;
}

void k_square_sum(const DevTables& T, u64* d, size_t d_comp, const Rows& a, size_t a_comp, void* stream) {
    ProfScope ps(T.prof, PK_TENSOR, 8.0 * T.N * a.rpg * (2.0 * a.ngroups + 3.0), stream);
    hipLaunchKernelGGL(square_sum_kernel, dim3((T.N + 255) / 256, a.rpg), dim3(256), 0, (hipStream_t)stream, T,
                       d, d_comp, a, a_comp);
}

// ---------------------------------------------------------- permutation
__global__ void permute_kernel(Rows out, Rows in, const int* perm, int N) {
    const int row = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    row_ptr(out, row, N)[i] = row_ptr(in, row, N)[perm[i]];
}

void k_permute(const DevTables& T, const Rows& out, const Rows& in, const int* perm, void* stream) {
    if (out.ngroups * out.rpg == 0) return;
    ProfScope ps(T.prof, PK_PERM, 16.0 * T.N * out.ngroups * out.rpg, stream);
    hipLaunchKernelGGL(permute_kernel, ew_grid(T, out), dim3(256), 0, (hipStream_t)stream, out, in, perm, T.N);
}

__global__ void permute_multi_kernel(Rows out, Rows in, PermList perms, int N) {
    const int row = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int G = row / out.rpg, r = row - G * out.rpg;
    const int* perm = perms.perm[G / perms.per];
    const u64* src = in.base + (size_t)(G % in.ngroups) * in.gstride + (size_t)r * N;
    row_ptr(out, row, N)[i] = src[perm[i]];
}

void k_permute_multi(const DevTables& T, const Rows& out, const Rows& in, const PermList& perms, void* stream) {
    if (out.ngroups * out.rpg == 0) return;
    if (perms.per < 1 || perms.n > kMaxKeys || (out.ngroups + perms.per - 1) / perms.per > perms.n ||
        in.rpg < out.rpg)
        launch_error("permutation batch: the permutation list does not cover the output groups");
    ProfScope ps(T.prof, PK_PERM, 16.0 * T.N * out.ngroups * out.rpg, stream);
    hipLaunchKernelGGL(permute_multi_kernel, ew_grid(T, out), dim3(256), 0, (hipStream_t)stream, out, in, perms,
                       T.N);
}

// --------------------------------------------------------- base conversion
// One thread per coefficient, K (the number of source primes) a template
// argument so the lifted sources stay in registers (a source row may also be
// copied unchanged to an output row: ModUp's own digit rows); the conversion constants
// (K x m products [D/d_s]_t and the target primes) are staged in LDS once per
// workgroup and read as broadcasts inside the product loop.
constexpr int kMaxConvSrc = 16;
constexpr int kMaxConvDst = 64;

// Products without carries: x_s = x1 2^32 + x0 (x1 < 2^30) and the constant
// [D/d_s]_t = h2 2^42 + h1 2^21 + h0 (21-bit limbs), so each of the six
// partial sums S_ij = sum_s x_i h_j stays below 2^57 for K <= 16 and is one
// v_mad_u64_u32 per product; the exact 128-bit sum is then
// sum_ij S_ij 2^(32 i + 21 j).  Targets below 2^42 have h2 = 0 and skip two.
template <int K, bool WIDE>
__device__ __forceinline__ unsigned __int128 conv_sum(const u32 (&x0)[K], const u32 (&x1)[K], const u64* hl,
                                                      const u32* h2, int m, int t) {
    u64 s00 = 0, s01 = 0, s02 = 0, s10 = 0, s11 = 0, s12 = 0;
#pragma unroll
    for (int s = 0; s < K; s++) {
        const u64 h = hl[s * m + t];
        const u32 a = (u32)h, b = (u32)(h >> 32);
        s00 += (u64)x0[s] * a;
        s01 += (u64)x0[s] * b;
        s10 += (u64)x1[s] * a;
        s11 += (u64)x1[s] * b;
        if (WIDE) {
            const u32 c = h2[s * m + t];
            s02 += (u64)x0[s] * c;
            s12 += (u64)x1[s] * c;
        }
    }
    unsigned __int128 v = s00;
    v += (unsigned __int128)s01 << 21;
    v += (unsigned __int128)s10 << 32;
    v += (unsigned __int128)s11 << 53;
    if (WIDE) {
        v += (unsigned __int128)s02 << 42;
        v += (unsigned __int128)s12 << 74;
    }
    return v;
}

template <int K>
__global__ void __launch_bounds__(256) base_convert_kernel(DevTables T, ConvTables C, u64* out, size_t og,
                                                           const u64* in, size_t ig, const u64* own_in,
                                                           size_t own_ig) {
    __shared__ u64 s_hl[K * kMaxConvDst];        // (h1 << 32) | h0
    __shared__ u32 s_h2[K * kMaxConvDst];
    __shared__ u64 s_q[kMaxConvDst], s_r64[kMaxConvDst], s_r64s[kMaxConvDst], s_one[kMaxConvDst],
        s_dmod[kMaxConvDst];
    __shared__ int s_row[kMaxConvDst];
    const int m = C.m;
    for (int e = threadIdx.x; e < K * m; e += blockDim.x) {
        const u64 h = C.hat[e];
        s_hl[e] = ((h >> 21) & 0x1FFFFF) << 32 | (h & 0x1FFFFF);
        s_h2[e] = (u32)(h >> 42);
    }
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
        s_q[t] = T.prime[C.dst_prime[t]].q;
        s_r64[t] = C.r64[t];
        s_r64s[t] = C.r64s[t];
        s_one[t] = C.ones[t];
        s_dmod[t] = C.dmod[t];
        s_row[t] = C.dst_row[t];
    }
    __syncthreads();
    const int g = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = T.N;
    if (i >= N) return;
    // blockIdx.z of gridDim.z takes one slice of the targets (more waves for
    // launches over few row groups)
    const int t0 = (m * (int)blockIdx.z) / (int)gridDim.z, t1 = (m * ((int)blockIdx.z + 1)) / (int)gridDim.z;
    u32 x0[K], x1[K];
    int nneg = 0;
#pragma unroll
    for (int s = 0; s < K; s++) {
        const u64 x = in[(size_t)g * ig + (size_t)C.src_row[s] * N + i];
        if (C.own_row && C.own_row[s] >= 0 && blockIdx.z == 0)
            out[(size_t)g * og + (size_t)C.own_row[s] * N + i] =
                own_in ? own_in[(size_t)g * own_ig + (size_t)C.src_row[s] * N + i] : x;
        const u64 d = T.prime[C.src_prime[s]].q;
        const u64 xh = mul_shoup(x, C.inv_hat[s], C.inv_hat_s[s], d);
        // centred: xh - d_s contributes xh * hat - D
        if (C.centered && xh > (d - 1) / 2) nneg++;
        x0[s] = (u32)xh;
        x1[s] = (u32)(xh >> 32);
    }
    u64* o = out + (size_t)g * og + i;
    for (int t = t0; t < t1; t++) {
        const u64 q = s_q[t];
        // the branch is uniform: every lane works on target t
        unsigned __int128 v = q >> 42 ? conv_sum<K, true>(x0, x1, s_hl, s_h2, m, t)
                                      : conv_sum<K, false>(x0, x1, s_hl, s_h2, m, t);
        // centred sources: - nneg D = + nneg (q - D mod q) modulo q, added
        // to the exact sum (nneg <= K, so it stays below 2^127)
        if (nneg) v += (unsigned __int128)(u64)nneg * (q - s_dmod[t]);
        // v mod q = (hi 2^64 mod q) + (lo mod q): two Shoup reductions
        const u64 hi = (u64)(v >> 64), lo = (u64)v;
        const u64 rl = lo - __umul64hi(lo, s_one[t]) * q;
        o[(size_t)s_row[t] * N] = add_mod(mul_shoup(hi, s_r64[t], s_r64s[t], q), rl >= q ? rl - q : rl, q);
    }
}

// Matrix-core form.  With x = sum_a d_a 256^a (balanced digits d_a in
// [-128, 127], read off as the bytes of (x + c) xor c, c = 0x80..80) and the
// constants H_(s,a),t = 2^(8a) [D/d_s]_t mod q_t split the same way into
// planes h_b, the int8 products C_b,t = sum_(s,a) d_(s,a) h_(s,a),t,b
// (|C| < 2^21) give V = sum_b C_b 2^(8b), congruent to sum_s xh_s [D/d_s]_t
// modulo q_t, so the reduced result is the VALU kernel's exactly.  One wave
// takes 16 coefficients per tile: A = 16 x 32 digits (four sources per MFMA
// step), B = 32 x 16 targets per plane, eight 16 x 16 int32 accumulators;
// every lane then folds the planes of 4 outputs.
typedef int v4i __attribute__((ext_vector_type(4)));
constexpr int kConvTiles = 8;            // 16-coefficient tiles per wave
constexpr u64 kDigitBias = 0x8080808080808080ull;
constexpr int kConvPlaneLds = 56 * 1024; // bytes of B operands one workgroup stages

template <int KS>
__global__ void __launch_bounds__(256) base_convert_mfma_kernel(DevTables T, ConvTables C, u64* out, size_t og,
                                                                const u64* in, size_t ig, const u64* own_in,
                                                                size_t own_ig) {
    extern __shared__ u64 sB[];          // [ntb][KS][8][64]
    __shared__ u64 s_q[kMaxConvDst], s_mu[kMaxConvDst], s_c48[kMaxConvDst], s_c48s[kMaxConvDst],
        s_dmod[kMaxConvDst];
    __shared__ int s_bits[kMaxConvDst], s_row[kMaxConvDst];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int quad = lane >> 4, col = lane & 15;
    const int g = blockIdx.y;
    const int N = T.N;
    const int m = C.m, ntb = C.ntb;
    for (int e = threadIdx.x; e < ntb * KS * 8 * 64; e += blockDim.x) sB[e] = C.bfrag[e];
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
        const PrimeInfo P = T.prime[C.dst_prime[t]];
        s_q[t] = P.q;
        s_mu[t] = P.mu;
        s_bits[t] = P.bits;
        s_c48[t] = C.c48[t];
        s_c48s[t] = C.c48s[t];
        s_dmod[t] = C.dmod[t];
        s_row[t] = C.dst_row[t];
    }
    __syncthreads();
    for (int tile = 0; tile < kConvTiles; tile++) {
        const int base = ((blockIdx.x * 4 + wave) * kConvTiles + tile) * 16;
        if (base >= N) break;   // whole wave
        // A operand: coefficient base + col, sources 4 ks + quad
        long afr[KS];
        int neg = 0;
#pragma unroll
        for (int ks = 0; ks < KS; ks++) {
            const int s = 4 * ks + quad;
            u64 x = 0;
            if (s < C.k) {
                const u64 v = in[(size_t)g * ig + (size_t)C.src_row[s] * N + base + col];
                if (C.own_row && C.own_row[s] >= 0)
                    out[(size_t)g * og + (size_t)C.own_row[s] * N + base + col] =
                        own_in ? own_in[(size_t)g * own_ig + (size_t)C.src_row[s] * N + base + col] : v;
                const u64 d = T.prime[C.src_prime[s]].q;
                x = mul_shoup(v, C.inv_hat[s], C.inv_hat_s[s], d);
                if (C.centered && x > (d - 1) / 2) neg++;
            }
            afr[ks] = (long)((x + kDigitBias) ^ kDigitBias);
        }
        int nneg[4] = {0, 0, 0, 0};
        if (C.centered) {
            neg += __shfl_xor(neg, 16);
            neg += __shfl_xor(neg, 32);
#pragma unroll
            for (int r = 0; r < 4; r++) nneg[r] = __shfl(neg, 4 * quad + r);
        }
        for (int tb = 0; tb < ntb; tb++) {
            v4i acc[8];
#pragma unroll
            for (int b = 0; b < 8; b++) acc[b] = v4i{0, 0, 0, 0};
            const u64* bt = sB + (size_t)tb * KS * 8 * 64;
#pragma unroll
            for (int ks = 0; ks < KS; ks++)
#pragma unroll
                for (int b = 0; b < 8; b++)
                    acc[b] = __builtin_amdgcn_mfma_i32_16x16x32_i8(afr[ks], (long)bt[(ks * 8 + b) * 64 + lane],
                                                                   acc[b], 0, 0, 0);
            const int t = tb * 16 + col;
            if (t >= m) continue;
            PrimeInfo P;
            P.q = s_q[t];
            P.mu = s_mu[t];
            P.bits = s_bits[t];
            const u64 c48 = s_c48[t], c48s = s_c48s[t];
            u64* o = out + (size_t)g * og + (size_t)s_row[t] * N + base + 4 * quad;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int p0 = acc[0][r] + acc[1][r] * 256;
                const int p1 = acc[2][r] + acc[3][r] * 256;
                const int p2 = acc[4][r] + acc[5][r] * 256;
                const int p3 = acc[6][r] + acc[7][r] * 256;
                const int64_t X = (int64_t)p0 + (int64_t)p1 * 65536 + (int64_t)p2 * 4294967296ll;
                u64 rx = reduce64(X < 0 ? (u64)(-X) : (u64)X, P);
                if (X < 0 && rx) rx = P.q - rx;
                const u64 p3m = p3 < 0 ? P.q - (u64)(-(int64_t)p3) : (u64)p3;
                u64 res = add_mod(rx, mul_shoup(p3m, c48, c48s, P.q), P.q);
                for (int k = 0; k < nneg[r]; k++) res = sub_mod(res, s_dmod[t], P.q);
                o[r] = res;
            }
        }
    }
}

template <int KS>
static void launch_base_convert_mfma(const DevTables& T, const ConvTables& C, u64* out, size_t og, const u64* in,
                                     size_t ig, int ngroups, const u64* own_in, size_t own_ig, hipStream_t st) {
    if (C.nks == KS) {
        const int per_block = 4 * kConvTiles * 16;
        const size_t lds = (size_t)C.ntb * KS * 8 * 64 * sizeof(u64);
        hipLaunchKernelGGL(base_convert_mfma_kernel<KS>, dim3((T.N + per_block - 1) / per_block, ngroups),
                           dim3(256), lds, st, T, C, out, og, in, ig, own_in, own_ig);
    } else if constexpr (KS < kMaxConvSrc / 4) {
        launch_base_convert_mfma<KS + 1>(T, C, out, og, in, ig, ngroups, own_in, own_ig, st);
    }
}

template <int K>
static void launch_base_convert(const DevTables& T, const ConvTables& C, u64* out, size_t og, const u64* in,
                                size_t ig, int ngroups, int split, const u64* own_in, size_t own_ig,
                                hipStream_t st) {
    if (C.k == K)
        hipLaunchKernelGGL(base_convert_kernel<K>, dim3((T.N + 255) / 256, ngroups, split), dim3(256), 0, st, T, C,
                           out, og, in, ig, own_in, own_ig);
    else if constexpr (K < kMaxConvSrc)
        launch_base_convert<K + 1>(T, C, out, og, in, ig, ngroups, split, own_in, own_ig, st);
}

static bool conv_planes_fit(const DevTables& T, const ConvTables& C) {
    return C.bfrag && T.N % 16 == 0 && (size_t)C.ntb * C.nks * 8 * 64 * sizeof(u64) <= (size_t)kConvPlaneLds;
}

// variant 0: VALU kernel; 1: matrix-core kernel (when its tables exist);
// 2, 3: VALU kernel with the targets split over 2 or 4 threads per coefficient
static const char* const kConvVariants[] = {"valu", "mfma", "valu/split2", "valu/split4"};
static void conv_launch(const DevTables& T, const ConvTables& C, u64* out, size_t og, const u64* in, size_t ig,
                        int ngroups, int variant, hipStream_t st, const u64* own_in = nullptr, size_t own_ig = 0) {
    if (variant == 1 && conv_planes_fit(T, C))
        launch_base_convert_mfma<1>(T, C, out, og, in, ig, ngroups, own_in, own_ig, st);
    else
        launch_base_convert<1>(T, C, out, og, in, ig, ngroups, variant == 2 ? 2 : variant == 3 ? 4 : 1, own_in,
                               own_ig, st);
}

// ------------------------------------------------------------- autotuner
// Interchangeable implementations of one operation (identical results) are
// timed on scratch data of the launch's shape the first time the shape is
// met while tuning is enabled, outside graph capture; the fastest is kept
// for the process (and can be saved and loaded).  A candidate whose output
// differs from the default's in any word is rejected.
namespace {
struct TuneEntry {
    int choice = 0;
    std::vector<std::string> names;
    std::vector<double> us;      // best time per candidate (microseconds), < 0: rejected
};
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;
int g_tune_on = -1;
thread_local int g_tune_suspended = 0;

bool tuning_on() {
    if (g_tune_suspended > 0) return false;
    if (g_tune_on < 0) {
        const char* e = std::getenv("HS_TUNE");
        g_tune_on = (e && std::string(e) == "1") ? 1 : 0;
    }
    return g_tune_on == 1;
}

__global__ void tune_fill_kernel(u64* p, size_t n, u64 seed) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    u64 z = (i + 1) * 0x9E3779B97F4A7C15ull + seed;    // SplitMix64 finaliser
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    p[i] = (z ^ (z >> 31)) & ((1ull << 39) - 1);        // below every prime
}

__global__ void tune_diff_kernel(const u64* a, const u64* b, size_t n, unsigned* bad) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && a[i] != b[i]) atomicAdd(bad, 1u);
}

void tune_fill(u64* p, size_t n, u64 seed, hipStream_t st) {
    if (n) hipLaunchKernelGGL(tune_fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, seed);
}

// Times `launch(c, in, out)` for every candidate; in-place candidates
// (out == in) get the input restored before each run.
int tune_run(const std::string& key, const std::vector<std::string>& names, const std::vector<bool>& ok,
             size_t in_words, size_t out_words, bool inplace, hipStream_t st,
             const std::function<void(int, const u64*, u64*)>& launch) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return 0;
    if (hipStreamSynchronize(st) != hipSuccess) return 0;
    u64 *in = nullptr, *pristine = nullptr, *out = nullptr, *ref = nullptr;
    unsigned* bad = nullptr;
    auto cleanup = [&] {
        (void)hipStreamSynchronize(st);
        for (void* p : {(void*)in, (void*)pristine, (void*)out, (void*)ref, (void*)bad})
            if (p) (void)hipFree(p);
    };
    const size_t ow = inplace ? in_words : out_words;
    if (hipMalloc(&in, in_words * 8) != hipSuccess || hipMalloc(&ref, ow * 8) != hipSuccess ||
        hipMalloc(&bad, sizeof(unsigned)) != hipSuccess ||
        (inplace ? hipMalloc(&pristine, in_words * 8) : hipMalloc(&out, out_words * 8)) != hipSuccess) {
        (void)hipGetLastError();
        cleanup();
        return 0;    // no room to tune: keep the default
    }
    tune_fill(in, in_words, 0x5eed, st);
    if (inplace) (void)hipMemcpyAsync(pristine, in, in_words * 8, hipMemcpyDeviceToDevice, st);
    u64* dst = inplace ? in : out;
    auto prepare = [&] {
        if (inplace) (void)hipMemcpyAsync(in, pristine, in_words * 8, hipMemcpyDeviceToDevice, st);
        else tune_fill(out, out_words, 0, st);
    };
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    TuneEntry E;
    E.names = names;
    E.us.assign(names.size(), -1.0);
    for (size_t c = 0; c < names.size(); c++) {
        if (!ok[c]) continue;
        double best = 1e30;
        for (int rep = 0; rep < 4; rep++) {
            prepare();
            (void)hipEventRecord(e0, st);
            launch((int)c, in, dst);
            (void)hipEventRecord(e1, st);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (rep > 0) best = std::min(best, 1e3 * ms);    // the first run warms caches
        }
        if (c == 0) {
            (void)hipMemcpyAsync(ref, dst, ow * 8, hipMemcpyDeviceToDevice, st);
        } else {
            unsigned nb = 0;
            (void)hipMemsetAsync(bad, 0, sizeof(unsigned), st);
            hipLaunchKernelGGL(tune_diff_kernel, dim3((unsigned)((ow + 255) / 256)), dim3(256), 0, st, dst, ref, ow,
                               bad);
            (void)hipMemcpyAsync(&nb, bad, sizeof(unsigned), hipMemcpyDeviceToHost, st);
            (void)hipStreamSynchronize(st);
            if (nb) continue;    // not interchangeable: rejected
        }
        E.us[c] = best;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    cleanup();
    for (size_t c = 0; c < names.size(); c++)
        if (E.us[c] >= 0 && (E.us[E.choice] < 0 || E.us[c] < E.us[E.choice])) E.choice = (int)c;
    if (std::getenv("HS_TRACE")) {
        std::fprintf(stderr, "[hs] tune %s:", key.c_str());
        for (size_t c = 0; c < names.size(); c++) std::fprintf(stderr, " %s=%.1fus", names[c].c_str(), E.us[c]);
        std::fprintf(stderr, " -> %s\n", names[E.choice].c_str());
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = E;
    return E.choice;
}

// decided variant for `key`, or -1 when the shape has not been tuned
int tune_lookup(const std::string& key) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(key);
    return it == g_tune.end() ? -1 : it->second.choice;
}

int pow2_bucket(int x) {
    int b = 1;
    while (b < x) b <<= 1;
    return b;
}
}  // namespace

int tune_conv(const DevTables& T, const ConvTables& C, size_t og, size_t ig, int ngroups, hipStream_t st) {
    const std::string key = "conv N=" + std::to_string(T.N) + " k=" + std::to_string(C.k) + " m=" +
                            std::to_string(C.m) + " groups=" + std::to_string(pow2_bucket(ngroups)) +
                            (C.centered ? " centred" : "");
    const int v = tune_lookup(key);
    if (v >= 0 || !tuning_on()) return v < 0 ? 0 : v;
    const int gq = pow2_bucket(ngroups);
    return tune_run(key, {kConvVariants, kConvVariants + 4}, {true, conv_planes_fit(T, C), C.m >= 4, C.m >= 8},
                    (size_t)gq * ig, (size_t)gq * og, false, st,
                    [&](int c, const u64* in, u64* out) { conv_launch(T, C, out, og, in, ig, gq, c, st); });
}

int tune_ntt16(const DevTables& T, const Rows& x, bool inverse, hipStream_t st, const NttSkip* skip) {
    // a skipping launch tunes over whole groups of its digit pattern
    const int gq = skip && skip->per ? ((pow2_bucket(x.ngroups) + skip->per - 1) / skip->per) * skip->per
                                     : pow2_bucket(x.ngroups);
    const std::string key = "ntt N=" + std::to_string(T.N) + " rows=" + std::to_string(x.rpg) + " groups=" +
                            std::to_string(gq) + (inverse ? " inverse" : " forward") +
                            (skip && skip->per ? " skip-own-digit" : "");
    const int v = tune_lookup(key);
    if (v >= 0 || !tuning_on()) return v < 0 ? 0 : v;
    const size_t words = (size_t)gq * x.rpg * T.N;
    return tune_run(key, {kNttVariants, kNttVariants + 8},
                    {true, true, gq > kNttGroupBatch, gq > kNttGroupBatch, true, true, gq > kNttGroupBatch,
                     gq > kNttGroupBatch},
                    words, 0, true, st,
                    [&](int c, const u64*, u64* buf) {
                        Rows r = x;
                        r.base = buf;
                        r.gstride = (size_t)x.rpg * T.N;
                        r.ngroups = gq;
                        ntt16_launch(T, r, r, inverse, c, st, nullptr, skip ? *skip : NttSkip());
                    });
}

void tune_enable(bool on) { g_tune_on = on ? 1 : 0; }

void tune_suspend(bool on) { g_tune_suspended += on ? 1 : -1; }

void tune_clear() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

// one entry per line: {"key": "...", "choice": "...", "us": {"name": t, ...}}
std::string tune_dump() {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::string s;
    char buf[64];
    for (auto& kv : g_tune) {
        s += "{\"key\": \"" + kv.first + "\", \"choice\": \"" + kv.second.names[kv.second.choice] + "\", \"us\": {";
        for (size_t c = 0; c < kv.second.names.size(); c++) {
            std::snprintf(buf, sizeof(buf), "%.2f", kv.second.us[c]);
            s += (c ? ", \"" : "\"") + kv.second.names[c] + "\": " + buf;
        }
        s += "}}\n";
    }
    return s;
}

// reads lines written by tune_dump; returns the number of entries taken
int tune_load(const std::string& text) {
    int n = 0;
    size_t pos = 0;
    while (pos < text.size()) {
        size_t eol = text.find('\n', pos);
        if (eol == std::string::npos) eol = text.size();
        const std::string line = text.substr(pos, eol - pos);
        pos = eol + 1;
        auto field = [&](const std::string& name) -> std::string {
            const std::string tag = "\"" + name + "\": \"";
            size_t a = line.find(tag);
            if (a == std::string::npos) return "";
            a += tag.size();
            size_t b = line.find('"', a);
            return b == std::string::npos ? "" : line.substr(a, b - a);
        };
        const std::string key = field("key"), choice = field("choice");
        if (key.empty() || choice.empty()) continue;
        std::vector<std::string> names;
        if (key.rfind("conv", 0) == 0) names = {kConvVariants, kConvVariants + 4};
        else if (key.rfind("ntt", 0) == 0)
            names = {kNttVariants, kNttVariants + 8};
        TuneEntry E;
        E.names = names;
        E.us.assign(names.size(), -1.0);
        E.choice = -1;
        for (size_t c = 0; c < names.size(); c++)
            if (names[c] == choice) E.choice = (int)c;
        if (E.choice < 0) continue;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = E;
        n++;
    }
    return n;
}

void k_base_convert(const DevTables& T, const ConvTables& C, u64* out, size_t out_gstride, const u64* in,
                    size_t in_gstride, int ngroups, void* stream, const u64* own_in, size_t own_gstride) {
    if (ngroups == 0 || C.m == 0) return;
    if (C.k < 1 || C.k > kMaxConvSrc || C.m > kMaxConvDst)
        launch_error("base conversion: source or target count out of range");
    const int variant = tune_conv(T, C, out_gstride, in_gstride, ngroups, (hipStream_t)stream);
    ProfScope ps(T.prof, PK_CONV, 8.0 * T.N * ngroups * (double)(C.k + C.m), stream);
    conv_launch(T, C, out, out_gstride, in, in_gstride, ngroups, variant, (hipStream_t)stream, own_in, own_gstride);
}

// centred lift: v = x if x <= (q_s - 1)/2 else x - q_s, reduced mod each row's prime
__global__ void lift_centered_kernel(DevTables T, Rows out, const u64* in, size_t ig, int src_prime) {
    const int row = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = T.N;
    if (i >= N) return;
    const int g = row / out.rpg;
    const int r = row - g * out.rpg;
    const PrimeInfo P = T.prime[prime_of(out, r)];
    row_ptr(out, row, N)[i] = lift_centred(in[(size_t)g * ig + i], T.prime[src_prime].q, P);
}

void k_lift_centered(const DevTables& T, const Rows& out, const u64* in, size_t in_gstride, int src_prime,
                     void* stream) {
    if (out.ngroups * out.rpg == 0) return;
    ProfScope ps(T.prof, PK_LIFT, 8.0 * T.N * out.ngroups * (out.rpg + 1.0), stream);
    hipLaunchKernelGGL(lift_centered_kernel, ew_grid(T, out), dim3(256), 0, (hipStream_t)stream, T, out, in,
                       in_gstride, src_prime);
}

// ------------------------------------------------------ key inner product
// ext:  [ncts][beta][E][N]   (E = nq_level + alpha extended rows)
// key:  [beta][2][key_rows][N]  (rows = all Q primes then all P primes)
// acc:  [ncts][2][E][N]
constexpr int kMaxDigits = 16;

template <int B>
__global__ void __launch_bounds__(256) key_inner_kernel(DevTables T, u64* acc, const u64* ext, KeyList keys,
                                                        int E, int nql, int key_rows, int key_nq) {
    const int r = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int N = T.N;
    if (i >= N) return;
    const int kr = r < nql ? r : key_nq + (r - nql);
    const PrimeInfo P = T.prime[kr];
    const u64 r64 = T.r64[kr];
    // each key is read once and applied to its block of ciphertexts
    for (int kk = 0; kk < keys.n; kk++) {
    const u64* key = keys.key[kk];
    u64 kb[B], ka[B];
#pragma unroll
    for (int j = 0; j < B; j++) {
        kb[j] = key[((size_t)(2 * j) * key_rows + kr) * N + i];
        ka[j] = key[((size_t)(2 * j + 1) * key_rows + kr) * N + i];
    }
    for (int g = kk * keys.per; g < (kk + 1) * keys.per; g++) {
        // exact sums of B <= 16 products below 2^122, reduced once
        unsigned __int128 s0 = 0, s1 = 0;
#pragma unroll
        for (int j = 0; j < B; j++) {
            const u64 x = ext[(((size_t)g * B + j) * E + r) * N + i];
            s0 += (unsigned __int128)x * kb[j];
            s1 += (unsigned __int128)x * ka[j];
        }
        acc[(((size_t)g * 2 + 0) * E + r) * N + i] = reduce_wide(s0, P, r64);
        acc[(((size_t)g * 2 + 1) * E + r) * N + i] = reduce_wide(s1, P, r64);
    }
    }
}

template <int B>
static void launch_key_inner(const DevTables& T, u64* acc, const u64* ext, const KeyList& keys, int beta, int E,
                             int nql, int key_rows, int key_nq, hipStream_t st) {
    if (beta == B)
        hipLaunchKernelGGL(key_inner_kernel<B>, dim3((T.N + 255) / 256, E), dim3(256), 0, st, T, acc, ext, keys, E,
                           nql, key_rows, key_nq);
    else if constexpr (B < kMaxDigits)
        launch_key_inner<B + 1>(T, acc, ext, keys, beta, E, nql, key_rows, key_nq, st);
}

void k_key_inner(const DevTables& T, u64* acc, const u64* ext, const KeyList& keys, int beta, int ext_rows,
                 int nq_level, int key_rows, int key_nq, void* stream) {
    if (beta < 1 || beta > kMaxDigits) launch_error("key inner product: digit count out of range");
    if (keys.n < 1 || keys.n > kMaxKeys || keys.per < 1) launch_error("key inner product: bad key list");
    // algorithmic bytes: each key once per launch, ext read and acc written per ciphertext
    const double ncts = (double)keys.n * keys.per;
    ProfScope ps(T.prof, PK_KEYIP, 8.0 * T.N * ext_rows * (2.0 * beta * keys.n + ncts * (beta + 2.0)), stream);
    launch_key_inner<1>(T, acc, ext, keys, beta, ext_rows, nq_level, key_rows, key_nq, (hipStream_t)stream);
}

// ------------------------------------------------------------- sampling
// uniform residues: row with prime index t uses domain (domain_base | t),
// coefficient i the Philox block at counter i; value = 128-bit block mod q
__global__ void sample_uniform_kernel(DevTables T, Rows out, u64 seed, u64 dbase) {
    EW_INDEX
    const int t = prime_of(out, r);
    u32 w[4];
    philox(seed, dbase | (u64)t, (u64)i, w);
    const u64 lo = ((u64)w[1] << 32) | w[0];
    const u64 hi = ((u64)w[3] << 32) | w[2];
    const u64 r64 = reduce64(0 - P.q, P);  // 2^64 mod q
    const u64 v = add_mod(mul_mod(reduce64(hi, P), r64, P), reduce64(lo, P), P.q);
    row_ptr(out, row, N)[i] = v;
}

void k_sample_uniform(const DevTables& T, const Rows& out, u64 seed, u64 domain_base, void* stream) {
    EW_LAUNCH(sample_uniform_kernel, out, seed, domain_base);
}

__global__ void sample_small_kernel(int64_t* out, int N, u64 seed, u64 domain, int kind, const u64* cdt, int ncdt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    u32 w[4];
    philox(seed, domain, (u64)i, w);
    int64_t v;
    if (kind == 0) {
        const u32 r = w[0] % 3u;
        v = r == 0 ? 0 : (r == 1 ? 1 : -1);
    } else {
        const u64 u = ((u64)w[1] << 32) | w[0];
        int k = 0;
        while (k < ncdt - 1 && u >= cdt[k]) k++;
        v = (w[2] & 1u) ? -(int64_t)k : (int64_t)k;
    }
    out[i] = v;
}

void k_sample_small(int64_t* out, int N, u64 seed, u64 domain, int kind, const u64* cdt, int ncdt, void* stream) {
    hipLaunchKernelGGL(sample_small_kernel, dim3((N + 255) / 256), dim3(256), 0, (hipStream_t)stream, out, N, seed,
                       domain, kind, cdt, ncdt);
}

__global__ void small_to_rows_kernel(DevTables T, Rows out, const int64_t* small) {
    EW_INDEX
    const int64_t v = small[i];
    u64 x;
    if (v >= 0) {
        x = reduce64((u64)v, P);
    } else {
        const u64 m = reduce64((u64)(-v), P);
        x = m ? P.q - m : 0;
    }
    row_ptr(out, row, N)[i] = x;
}

void k_small_to_rows(const DevTables& T, const Rows& out, const int64_t* small, void* stream) {
    EW_LAUNCH(small_to_rows_kernel, out, small);
}

// ------------------------------------------------------------ copy / zero
__global__ void copy_rows_kernel(Rows out, Rows in, int N) {
    const int row = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    row_ptr(out, row, N)[i] = row_ptr(in, row, N)[i];
}
__global__ void zero_rows_kernel(Rows out, int N) {
    const int row = blockIdx.y;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    row_ptr(out, row, N)[i] = 0;
}

void k_copy_rows(const DevTables& T, const Rows& out, const Rows& in, void* stream) {
    if (out.ngroups * out.rpg == 0) return;
    hipLaunchKernelGGL(copy_rows_kernel, ew_grid(T, out), dim3(256), 0, (hipStream_t)stream, out, in, T.N);
}

void k_zero_rows(const DevTables& T, const Rows& out, void* stream) {
    if (out.ngroups * out.rpg == 0) return;
    hipLaunchKernelGGL(zero_rows_kernel, ew_grid(T, out), dim3(256), 0, (hipStream_t)stream, out, T.N);
}

// ------------------------------------------------------------- encoding
// value = rint(scale * w) as an exact integer, reduced mod the row's prime
__device__ u64 double_to_residue(double v, const PrimeInfo& P) {
    const bool neg = v < 0;
    const double a = neg ? -v : v;
    u64 mag;
    if (a < 9.2e18) {
        mag = reduce64((u64)a, P);
    } else {
        int e;
        const double m = frexp(a, &e);                 // a = m 2^e, m in [0.5, 1)
        const u64 mant = (u64)ldexp(m, 53);            // exact 53-bit integer
        int sh = e - 53;                               // a = mant * 2^sh, sh > 0
        u64 p2 = 1, base = 2 % P.q;
        while (sh > 0) {
            if (sh & 1) p2 = mul_mod(p2, base, P);
            base = mul_mod(base, base, P);
            sh >>= 1;
        }
        mag = mul_mod(reduce64(mant, P), p2, P);
    }
    return (neg && mag) ? P.q - mag : mag;
}

__global__ void encode_real_kernel(DevTables T, Rows out, const double* w, size_t wg, double scale) {
    EW_INDEX
    const int g = row / out.rpg;
    const double v = rint(scale * w[(size_t)g * wg + i]);
    row_ptr(out, row, N)[i] = double_to_residue(v, P);
}

void k_encode_real(const DevTables& T, const Rows& out, const double* w, size_t w_gstride, double scale,
                   void* stream) {
    EW_LAUNCH(encode_real_kernel, out, w, w_gstride, scale);
}

// ------------------------------------------------ multiplier throughput probe
// Eight independent chains of v_mad_u64_u32 (32 x 32 + 64 -> 64) per lane:
// the rate of the instruction every 64-bit modular product here is built from.
__global__ void __launch_bounds__(256) mul_rate_kernel(u64* out, u64 seed, int iters) {
    u64 a[8];
#pragma unroll
    for (int c = 0; c < 8; c++) a[c] = seed + threadIdx.x * 17 + c * 131;
    const u32 b = (u32)(seed >> 3) | 1;
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int u = 0; u < 8; u++)
#pragma unroll
            for (int c = 0; c < 8; c++) a[c] = (u64)(u32)a[c] * b + a[c];
    }
    u64 r = 0;
#pragma unroll
    for (int c = 0; c < 8; c++) r ^= a[c];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = r;
}

double k_mul_rate(void* stream) {
    hipStream_t st = (hipStream_t)stream;
    const int blocks = 256 * 16, iters = 512;
    u64* d = nullptr;
    if (hipMalloc((void**)&d, sizeof(u64) * blocks * 256) != hipSuccess) return 0.0;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    hipLaunchKernelGGL(mul_rate_kernel, dim3(blocks), dim3(256), 0, st, d, 12345ull, iters);
    (void)hipEventRecord(e0, st);
    hipLaunchKernelGGL(mul_rate_kernel, dim3(blocks), dim3(256), 0, st, d, 12345ull, iters);
    (void)hipEventRecord(e1, st);
    (void)hipEventSynchronize(e1);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(d);
    return 64.0 * iters * (double)blocks * 256 / (ms * 1e-3) / 1e12;
}

}  // namespace hs
