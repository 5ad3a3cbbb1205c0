// Interface between the host runtime (built with g++) and the HIP kernels
// (built with hipcc for gfx950): plain structs and launch wrappers.
#pragma once
#include <string>
#include <cstdint>
#include <cstddef>

typedef uint64_t u64;
typedef uint32_t u32;

namespace hs {

// Modulus data for one prime q < 2^61.  Barrett: b = bit length of q,
// mu = floor(2^(2b) / q).
struct PrimeInfo {
    u64 q;
    u64 mu;
    int bits;
    int pad;
    u64 nq;   // 2^64 - q: a w - h q = a w + h nq (mod 2^64), one multiply-add chain
};

// Per-launch timing with HIP events (off unless enabled): each profiled
// launch wrapper records an event pair and its algorithmic bytes.
struct Profiler;
enum ProfKind { PK_NTT = 0, PK_KEYIP, PK_CONV, PK_TENSOR, PK_EW, PK_PERM, PK_LIFT, PK_OTHER, PK_COUNT };
Profiler* prof_create();
void prof_destroy(Profiler* p);
void prof_enable(Profiler* p, bool on);
bool prof_enabled(const Profiler* p);
// totals since the last call, per kind: [count, milliseconds, bytes]; syncs the events
void prof_collect(Profiler* p, double* out);

// Device-resident tables of one context (negacyclic NTT twiddles in
// bit-reversed order, with Shoup companions floor(w 2^64 / q)).
struct DevTables {
    const PrimeInfo* prime;   // [n_primes]
    const u64* tw;            // [n_primes][N]   psi^brv(k)
    const u64* tws;
    const u64* itw;           // [n_primes][N]   psi^-brv(k)
    const u64* itws;
    const u64* ninv;          // [n_primes][2]   N^-1 mod q, Shoup companion
    const u64* tw2;           // [n_primes][N][2] (psi^brv(k), Shoup companion) interleaved
    const u64* itw2;          // [n_primes][N][2] (psi^-brv(k), Shoup companion) interleaved
    const u64* r64;           // [n_primes]      2^64 mod q
    int logN;
    int N;
    Profiler* prof;           // optional launch profiler (host object)
};

// A set of rows: ngroups groups of rpg consecutive rows (N words each);
// group g starts gstride words after group g-1.  Row r of a group uses prime
// index q_off + r when r < nq, else p_base + (r - nq).
struct Rows {
    u64* base;
    int ngroups;
    int rpg;
    size_t gstride;
    int nq;
    int q_off;
    int p_base;
};

constexpr int kMaxRows = 64;
// Per-row constants (indexed by the row within its group), passed by value.
struct RowConsts {
    u64 c[kMaxRows];
    u64 cs[kMaxRows];
};

// Constants of one fast base conversion, k source rows -> m target rows of
// the same group: y_t = sum_i [x_i inv_hat_i]_{d_i} * hat[i][t] mod q_t.
struct ConvTables {
    const u64* inv_hat;     // [k]
    const u64* inv_hat_s;   // [k]
    const u64* hat;         // [k * m]
    const u64* hat_s;       // [k * m]
    const int* src_prime;   // [k]
    const int* dst_prime;   // [m]
    const int* src_row;     // [k] row offsets (within the input group)
    const int* dst_row;     // [m] row offsets (within the output group)
    const int* own_row;     // [k] output row that receives source s unchanged, or -1 (null: none)
    const u64* dmod;        // [m]  D mod q_t (centred conversion only)
    const u64* r64;         // [m]  2^64 mod q_t
    const u64* r64s;        // [m]  Shoup companion of r64
    const u64* ones;        // [m]  floor(2^64 / q_t): Shoup companion of 1
    int k;
    int m;
    int centered;           // 1: [x_i inv_hat_i] taken in (-d_i/2, d_i/2]
    // byte-plane form for the matrix cores (null when a prime is out of its
    // range): sources split into 8 signed base-256 digits, constants
    // 2^(8a) [D/d_s]_t mod q_t likewise, one MFMA operand per lane
    const u64* bfrag;       // [ntb][nks][8 planes][64 lanes]
    const u64* c48;         // [m] 2^48 mod q_t
    const u64* c48s;        // [m] Shoup companions
    int nks;                // ceil(k / 4): 32-deep MFMA steps (four sources)
    int ntb;                // ceil(m / 16): 16-target blocks
};

// Fixed device scratch of the allocation-free entry point (scratch.hip):
// kScratchBytes per device, looked up once per device at context creation
// (with the device current).  scratch_init returns 1 when the array's device
// address is known, -1 when the lookup failed; scratch_device_ptr returns
// that address (null before a successful lookup).
constexpr size_t kScratchBytes = (size_t)96 << 20;
int scratch_init(int device);
void* scratch_device_ptr(int device);

// Autotuner over interchangeable kernel variants (base conversion: VALU or
// matrix cores; N = 2^16 NTT: row order and launch batching).  Off unless
// enabled (or HS_TUNE=1); decisions are process-wide.
void tune_enable(bool on);
void tune_clear();                       // forget every decision (defaults again)
std::string tune_dump();                 // one JSON object per line
int tune_load(const std::string& text);  // entries taken
// while suspended (a counter: nested calls), shapes without a decision use the
// default kernel and nothing is timed (timing allocates scratch buffers)
void tune_suspend(bool on);

// Epilogue of a forward NTT of rows x (groups G = 0..ngroups-1, rows r of a
// group use primes q_off + r): instead of NTT(x), write
//   out_j[G / split][r] = (d_j[G / split][r] +) (a[G][r] - NTT(x)[G][r]) (c[r])
// with j = G mod split (split = 1 or 2: the two components of ModDown); the
// addend is taken where d_j is not null, the factor c where mul is set.
struct NttEpilogue {
    int split = 1;
    bool mul = true;
    u64* out[2] = {nullptr, nullptr};
    size_t out_gs[2] = {0, 0};
    const u64* a = nullptr;
    size_t a_gs = 0;
    const u64* d[2] = {nullptr, nullptr};
    size_t d_gs[2] = {0, 0};
    int g0 = 0;                  // group offset of a partial launch
    RowConsts c;
};

// ------------------------------------------------------------- launches
// All launches are asynchronous on `stream` (a hipStream_t).  A launch
// wrapper given arguments its kernel cannot serve raises the library's
// argument error (HS_E_ARG) through launch_error instead of returning with
// the output unwritten.
[[noreturn]] void launch_error(const char* what);
void k_ntt(const DevTables& T, const Rows& x, bool inverse, void* stream);
// measured v_mad_u64_u32 rate of the device (10^12 lane operations / s)
double k_mul_rate(void* stream);
// x = NTT(src) (or its inverse); src has x's shape and may be x itself
void k_ntt_from(const DevTables& T, const Rows& x, const Rows& src, bool inverse, void* stream);
// Rows of a ModUp extension that the N = 2^16 forward transform leaves out:
// group G (ciphertext-major, digit G mod per) skips rows [lo, hi) with
// lo = (G mod per) digit, hi = min(lo + digit, nql) (the digit's own rows,
// already in the NTT domain).  per = 0: no rows are skipped.
struct NttSkip {
    int per = 0;
    int digit = 0;
    int nql = 0;
};
void k_ntt_skip(const DevTables& T, const Rows& x, const NttSkip& skip, void* stream);
// Input of a forward NTT taken as the centred lift of one coefficient-domain
// row per group (base + G gs, prime src_prime) to each row's prime, instead
// of x's own rows (rescale: the dropped row lifted to every other prime).
struct NttLift {
    const u64* base = nullptr;
    size_t gs = 0;
    int src_prime = 0;
};
// forward NTT of x (or of the lift, when given) followed by the epilogue
// (x is left unspecified)
void k_ntt_epilogue(const DevTables& T, const Rows& x, const NttEpilogue& e, void* stream,
                    const NttLift* lift = nullptr);
void k_add(const DevTables& T, const Rows& out, const Rows& a, const Rows& b, void* stream);
void k_sub(const DevTables& T, const Rows& out, const Rows& a, const Rows& b, void* stream);
void k_neg(const DevTables& T, const Rows& out, const Rows& a, void* stream);
void k_mul(const DevTables& T, const Rows& out, const Rows& a, const Rows& b, void* stream);
// out = sum over t < nterms of a[t] * p[t] mod q: a[t] are groups x rows
// contiguous rows (rows = level + 1, Q primes from q_0), p[t] are rows
// plaintext rows broadcast over the groups
constexpr int kMaxMacTerms = 16;
void k_mul_plain_acc(const DevTables& T, u64* out, const u64* const* a, const u64* const* p, int nterms,
                     int groups, int rows, void* stream);
// One leaf of a polynomial evaluation in one launch per 16 terms:
// out[G][r] = sum_t a_t[G][r] * f_t(r) over rows r < rows of every group G
// (a_t keeps arows rows per group: reading the first `rows` is the drop to
// the output's level), f_t a plaintext row p[r] or, where p is null, the
// integer (neg ? -1 : 1) mant 2^e reduced modulo q_r.
struct LeafTerm {
    const u64* a;
    int arows;
    const u64* p;
    u64 mant;
    int e;
    int neg;
};
void k_leaf_mac(const DevTables& T, u64* out, int groups, int rows, const LeafTerm* terms, int nterms,
                void* stream);
void k_mul_add(const DevTables& T, const Rows& acc, const Rows& a, const Rows& b, void* stream);
void k_mul_row_const(const DevTables& T, const Rows& out, const Rows& a, const RowConsts& c, void* stream);
void k_add_row_const(const DevTables& T, const Rows& out, const Rows& a, const RowConsts& c, void* stream);
// out = (a - b) * c_row
void k_sub_mul_const(const DevTables& T, const Rows& out, const Rows& a, const Rows& b,
                     const RowConsts& c, void* stream);
// out = d + (a - b) * c_row
void k_add_sub_mul_const(const DevTables& T, const Rows& out, const Rows& d, const Rows& a,
                         const Rows& b, const RowConsts& c, void* stream);
// tensor product of ciphertext pairs: groups are ciphertexts; a, b have 2
// components (component stride = rows * N inside the group), d has 3.
void k_tensor(const DevTables& T, const Rows& d, const Rows& a, const Rows& b, size_t a_comp,
              size_t b_comp, size_t d_comp, void* stream);
// sum over the groups of a of a (x) a, written to one degree-2 ciphertext d
void k_square_sum(const DevTables& T, u64* d, size_t d_comp, const Rows& a, size_t a_comp,
                  void* stream);
void k_permute(const DevTables& T, const Rows& out, const Rows& in, const int* perm, void* stream);
// several automorphisms in one launch: output group G reads input group
// G mod in.ngroups through perm[G / per]
constexpr int kMaxKeys = 32;
struct PermList {
    const int* perm[kMaxKeys];
    int n;
    int per;
};
void k_permute_multi(const DevTables& T, const Rows& out, const Rows& in, const PermList& perms, void* stream);
// keys of a batched key switch: ciphertext g uses key[g / per]
struct KeyList {
    const u64* key[kMaxKeys];
    int n;
    int per;
};
// own rows (ConvTables::own_row) are copied from own_in (group stride
// own_gstride, same row indices as in) when it is given, else from in
void k_base_convert(const DevTables& T, const ConvTables& C, u64* out, size_t out_gstride,
                    const u64* in, size_t in_gstride, int ngroups, void* stream, const u64* own_in = nullptr,
                    size_t own_gstride = 0);
// centred lift of one row (prime src_prime, coefficient domain) of each
// group to the rows of `out` (coefficient domain)
void k_lift_centered(const DevTables& T, const Rows& out, const u64* in, size_t in_gstride,
                     int src_prime, void* stream);
// hybrid key-switching inner product: for each ciphertext g and extended row
// r: acc0 = sum_j ext[g][j][r] * key[j][0][kr(r)], acc1 likewise with key[j][1]
void k_key_inner(const DevTables& T, u64* acc, const u64* ext, const KeyList& keys, int beta, int ext_rows,
                 int nq_level, int key_rows, int key_nq, void* stream);
void k_sample_uniform(const DevTables& T, const Rows& out, u64 seed, u64 domain_base, void* stream);
// kind: 0 uniform ternary, 2 gaussian (cdt table in device memory)
void k_sample_small(int64_t* out, int N, u64 seed, u64 domain, int kind, const u64* cdt, int ncdt,
                    void* stream);
void k_small_to_rows(const DevTables& T, const Rows& out, const int64_t* small, void* stream);
void k_copy_rows(const DevTables& T, const Rows& out, const Rows& in, void* stream);
void k_zero_rows(const DevTables& T, const Rows& out, void* stream);
// out = round(scale * w) mod q_row for each row (w: N doubles per group)
void k_encode_real(const DevTables& T, const Rows& out, const double* w, size_t w_gstride,
                   double scale, void* stream);

}  // namespace hs
