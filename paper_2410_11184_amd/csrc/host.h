// Host runtime of the homomorphic Softmax library: parameter set, device
// tables, key material, ciphertext buffers and the homomorphic operations
// built from the kernels in kernels.hip.
#pragma once
#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "dev.h"

namespace hs {

typedef unsigned __int128 u128;

// Status codes (mirrors include/hs.h)
enum Status {
    OK = 0,
    E_ARG = -1,
    E_PARAM = -2,
    E_LEVEL = -3,
    E_SCALE = -4,
    E_KEY = -5,
    E_OOM = -6,
    E_DEVICE = -7,
    E_RANGE = -8,
    E_STATE = -9,
};

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HS_REQUIRE(cond, code, msg) \
    do {                            \
        if (!(cond)) throw ::hs::Error((code), (msg)); \
    } while (0)

// ------------------------------------------------------------ parameters
struct BootParams {
    int cts_levels = 0;      // coefficient-to-slot levels (0 = no bootstrapping)
    int evalmod_levels = 0;
    int stc_levels = 0;
    int K = 32;              // |I| bound of the modular reduction
    int double_angle = 3;
    int cos_degree = 63;
    int log_boot_scale = 50;
};

struct Params {
    int logN = 12;
    std::vector<int> q_bits;
    std::vector<int> p_bits;
    int digit = 2;
    int hamming = 0;
    double sigma = 3.2;
    int log_scale = 40;
    int user_top = 0;
    BootParams boot;
};

// --------------------------------------------------------------- memory
// Where a context's device memory comes from: the caller's callbacks (the
// C ABI's hs_ctx_create_ex; the Python binding passes torch's caching
// allocator) or, without them, hipMalloc / hipFree.  get returns null when
// the memory is not available.
struct DevAllocator {
    void* (*alloc_fn)(size_t bytes, void* stream, void* user) = nullptr;
    void (*free_fn)(void* p, size_t bytes, void* user) = nullptr;
    void* user = nullptr;
    void* stream = nullptr;
    void* get(size_t bytes) const;
    void put(void* p, size_t bytes) const;
};

// Device memory arena: chunks obtained from hipMalloc (8 GiB, or the request
// rounded to 1 GiB when larger) and sub-allocated best-fit in 256-byte units,
// with neighbouring free blocks coalesced.  Chunks are kept until the context
// ends, so steady-state work allocates without hipMalloc / hipFree (which
// synchronise the device).  Every use is on the context's one stream, so a
// freed block may be reused at once.
class Pool {
public:
    void* alloc(size_t bytes);
    void free(void* p);
    void release_all();
    size_t trim(size_t bytes);   // release wholly free chunks until >= bytes freed
    // a fixed region instead of hipMalloc chunks: the pool never grows (an
    // allocation that does not fit raises E_OOM) and never frees it
    void adopt(void* base, size_t bytes);
    // chunks come from (and go back to) this source instead of hipMalloc
    void set_source(const DevAllocator* d) { src_ = d; }
    bool owns(const void* p) const { return live_.count(const_cast<void*>(p)) != 0; }
    size_t bytes_in_use() const { return in_use_; }
    size_t bytes_reserved() const { return reserved_; }
    ~Pool();

private:
    struct Chunk {
        char* base = nullptr;
        size_t size = 0;
        std::map<size_t, size_t> free_;   // offset -> size
    };
    std::vector<Chunk> chunks_;
    std::multimap<size_t, std::pair<int, size_t>> by_size_;   // size -> (chunk, offset)
    std::map<void*, std::pair<int, size_t>> live_;            // pointer -> (chunk, size)
    size_t in_use_ = 0, reserved_ = 0;
    bool fixed_ = false;
    const DevAllocator* src_ = nullptr;
    void* get_chunk(size_t bytes);
    void put_chunk(void* p, size_t bytes);
    void add_free(int c, size_t off, size_t size);
    void remove_free(int c, size_t off, size_t size);
};

struct DevBuf {
    u64* p = nullptr;
    size_t words = 0;
};

// A batch of m ciphertexts with the same level and component count, stored
// densely as [m][ncomp][level+1][N] 64-bit residues (NTT domain).
struct Ct {
    u64* d = nullptr;
    int m = 1;
    int ncomp = 2;
    int level = 0;
    double scale = 1.0;
    size_t comp_words(int N) const { return (size_t)(level + 1) * N; }
    size_t ct_words(int N) const { return (size_t)ncomp * (level + 1) * N; }
};

struct ConvDev {
    ConvTables t;
    std::vector<void*> bufs;
};

struct Context;

// Homomorphic operations counted per level (ciphertext equivalents: one
// degree-1 ciphertext = 1), for cost models of other implementations of the
// same schedule: key switches, tensor products (squares included), rescales,
// plaintext or constant products, additions.
enum OpKind { OC_KS = 0, OC_TENSOR, OC_RESCALE, OC_PTMUL, OC_ADD, OC_COUNT };

// Owned ciphertext handle (frees its buffer through the context's pool).
struct CtHandle {
    Context* ctx = nullptr;
    Ct ct;
    ~CtHandle();
};

struct Context {
    Params prm;
    int N = 0, logN = 0;
    std::vector<u64> primes;     // Q primes then P primes
    int nq = 0, np = 0;
    int L = 0;                   // top level (nq - 1)
    int dnum = 0;
    std::vector<u64> psi;
    DevTables T{};
    void* stream = nullptr;
    int device = 0;
    DevAllocator da;             // source of every device allocation of the context
    Pool pool;
    // arena that alloc_words draws from: `pool`, or a captured Softmax
    // schedule's own arena while it is being recorded
    Pool* cur = &pool;
    bool capturing = false;      // host-device copies and syncs are refused while set
    // captured Softmax schedules alive on this context: their graphs hold the
    // device addresses of the keys, so key generation is refused meanwhile
    int live_plans = 0;
    std::vector<PrimeInfo> pinfo;
    u64 P_mod[kMaxRows];         // P mod q_i for Q primes
    // key material
    bool have_keys = false;
    u64 key_seed = 0;
    std::vector<int64_t> s_coeff;
    u64* s_ntt = nullptr;        // [nq + np][N]
    u64* pk = nullptr;           // [2][nq][N]
    std::map<int, u64*> keys;    // key id -> [dnum][2][nq + np][N]
    u64* cdt = nullptr;
    int ncdt = 0;
    std::vector<u64> cdt_host;
    std::map<std::pair<int, int>, ConvDev> modup;   // (level, digit)
    std::map<int, ConvDev> moddown;                 // level
    std::map<int, int*> perms;                      // galois element -> device perm
    std::map<int, u64*> monomials;                  // k -> NTT of X^k over all Q primes
    void* boot = nullptr;                           // bootstrapping tables (boot.cpp), built on first use
    std::map<int, double*> mask_coeffs;             // L -> coefficients of the slot mask [0, L)
    // NTT-domain plaintexts rint(scale * mask) over rows 0..level, keyed by
    // (mask, level, exact scale): a Softmax schedule meets the same ones in
    // every job; kept up to kMaskCacheBytes
    std::map<std::tuple<const double*, int, double>, u64*> mask_pts;
    size_t mask_pts_bytes = 0;
    static constexpr size_t kMaskCacheBytes = (size_t)8 << 30;
    std::vector<void*> owned;                       // device tables
    std::map<void*, size_t> raw_sizes;              // raw_alloc'd blocks and their sizes
    std::vector<double> tw_cos, tw_sin;             // encoding twiddles, [2N]
    double opc[OC_COUNT][kMaxRows] = {};            // operation counts by level
    void count(int kind, int level, double n) {
        if (level >= 0 && level < kMaxRows) opc[kind][level] += n;
    }

    Context(const Params& p, int device, void* stream, const DevAllocator* alloc = nullptr);
    // A context on another stream that reads the key material and device
    // tables of `parent` (borrowed, never freed here); it builds its own
    // conversion tables, permutations, bootstrap plaintexts and any key it
    // adds (the same words as the parent's: the same seed).  The parent must
    // outlive it; key generation is refused on both while it lives.
    Context(Context& parent, void* stream);
    Context* parent_ctx = nullptr;
    int live_clones = 0;             // guarded by clone_mutex()
    bool destroy_pending = false;    // destroyed by its owner while clones lived
    std::vector<int> borrowed_keys;  // key ids whose device memory belongs to the parent
    ~Context();
    void release();   // returns every device block (destructor; failed construction)
    void init();      // the constructor's work

    // helpers
    u64 q(int i) const { return primes[i]; }
    Rows rows(u64* base, int ngroups, int rpg, size_t gstride, int q_off = 0) const {
        return Rows{base, ngroups, rpg, gstride, rpg, q_off, nq};
    }
    Rows ext_rows(u64* base, int ngroups, int nql, size_t gstride) const {
        return Rows{base, ngroups, nql + np, gstride, nql, 0, nq};
    }
    Rows p_rows(u64* base, int ngroups, size_t gstride) const {
        return Rows{base, ngroups, np, gstride, 0, 0, nq};
    }
    Rows ct_rows(const Ct& c) const {  // all rows of all components of all cts
        return Rows{c.d, c.m * c.ncomp, c.level + 1, (size_t)(c.level + 1) * N, c.level + 1, 0, nq};
    }
    Rows comp_rows(const Ct& c, int comp) const {
        return Rows{c.d + (size_t)comp * c.comp_words(N), c.m, c.level + 1, c.ct_words(N), c.level + 1, 0, nq};
    }
    u64* alloc_words(size_t w) { return (u64*)cur->alloc(w * sizeof(u64)); }
    void free_words(u64* p) {
        if (cur != &pool && cur->owns(p)) cur->free(p);
        else pool.free(p);
    }
    void sync();
    void upload(void* dst, const void* src, size_t bytes);
    void download(void* dst, const void* src, size_t bytes);
    void* dev_table(const void* host, size_t bytes);   // permanent device copy
    void* persistent_alloc(size_t bytes, const char* what);  // device memory owned until the context ends
    void* raw_alloc(size_t bytes, const char* what);          // from da, trimming the pool's cache if needed
    void raw_free(void* p);

    const ConvDev& modup_tables(int level, int j);
    const ConvDev& moddown_tables(int level);
    const int* perm(int g);
    RowConsts shoup_consts(const std::vector<u64>& vals, int q_off, bool p_part = false) const;
};

// Key material lives as long as the context: while in scope, allocations come
// from the context's own arena even when a captured schedule's arena is active.
// Bookkeeping of clones (live_clones, destroy_pending) across threads.
std::mutex& clone_mutex();
// Delete a context, or only mark it when clones still read its keys: then
// the last clone's release deletes it.
void destroy_context(Context* c);

struct ContextArena {
    Context& c;
    Pool* prev;
    explicit ContextArena(Context& cc) : c(cc), prev(cc.cur) { c.cur = &c.pool; }
    ~ContextArena() { c.cur = prev; }
};

// ----------------------------------------------------------- arithmetic
u64 mulmod_h(u64 a, u64 b, u64 q);
u64 powmod_h(u64 a, u64 e, u64 q);
u64 invmod_h(u64 a, u64 q);
u64 shoup_h(u64 w, u64 q);
int galois_rot(int r, int N);
void boot_release(Context* c);

// --------------------------------------------------------- ciphertexts
Ct ct_alloc(Context& c, int m, int ncomp, int level);
void ct_free(Context& c, Ct& ct);
Ct ct_copy(Context& c, const Ct& a);
Ct ct_drop(Context& c, const Ct& a, int level);          // copy to a lower level
Ct ct_slice(Context& c, const Ct& a, int first, int count);
Ct ct_gather(Context& c, const std::vector<const Ct*>& parts);

// ---------------------------------------------------- keys / encoding
void keygen(Context& c, u64 seed);
void add_galois_key(Context& c, int g);
bool has_key(const Context& c, int id);
void special_fft_inverse(const Context& c, std::vector<double>& re, std::vector<double>& im);
void special_fft(const Context& c, std::vector<double>& re, std::vector<double>& im);
// encode a slot vector (n = N/2 complex values) into NTT-domain rows 0..level
void encode_to(Context& c, u64* out_rows, const double* re, const double* im, int level, double scale);
Ct encrypt(Context& c, const u64* pt_rows, int level, double scale, u64 seed);
void decrypt_decode(Context& c, const Ct& a, int index, double* re, double* im);
std::vector<double> decrypt_coeffs_double(Context& c, const Ct& a, int index);

// --------------------------------------------------------------- ops
void op_add_inplace(Context& c, Ct& a, const Ct& b);         // a += b (b may have m = 1)
void op_sub_inplace(Context& c, Ct& a, const Ct& b);
Ct op_add(Context& c, const Ct& a, const Ct& b);
Ct op_sub(Context& c, const Ct& a, const Ct& b);
void op_neg_inplace(Context& c, Ct& a);
void op_mul_int_inplace(Context& c, Ct& a, long long k);     // scale unchanged
void op_mul_residues_inplace(Context& c, Ct& a, const std::vector<u64>& res);
void op_add_const_inplace(Context& c, Ct& a, double v);       // adds rint(v * scale)
Ct op_mul_const(Context& c, const Ct& a, double v, double target_scale); // const mult + rescale
Ct op_mul_plain(Context& c, const Ct& a, const u64* pt, double pt_scale, bool rescale);
Ct op_tensor(Context& c, const Ct& a, const Ct& b);
Ct op_square_sum(Context& c, const Ct& a);                 // sum_g a_g (x) a_g
Ct op_square_sum_jobs(Context& c, const Ct& a, int jobs);  // one such sum per group of a.m / jobs ciphertexts
Ct op_relin(Context& c, const Ct& d);
Ct op_rescale(Context& c, const Ct& a);
Ct op_mult(Context& c, const Ct& a, const Ct& b);            // tensor, relin, rescale
// the same product of two ciphertexts of one level written to out (rows of
// the output level); returns the output scale
double op_mult_into(Context& c, const Ct& a, const Ct& b, bool rescale, u64* out);
Ct op_apply_galois(Context& c, const Ct& a, int g);
Ct op_rotate(Context& c, const Ct& a, int r);
Ct op_conjugate(Context& c, const Ct& a);
// rotations of a by every r in rots with one shared ModUp (values as op_rotate)
// rotations of a by every r in rots (none a multiple of the slot count) with
// one ModUp: one batch of rots.size() * a.m ciphertexts, rotation-major
Ct op_rotate_hoisted_batch(Context& c, const Ct& a, const std::vector<int>& rots);
// block i of `per` ciphertexts of a through Galois element gal[i]
Ct op_galois_batch(Context& c, const Ct& a, const std::vector<int>& gal, int per);
Ct op_mod_raise(Context& c, const Ct& a, int level);
Ct op_mul_monomial(Context& c, const Ct& a, int k);
// ModUp of the polynomials d (level l, NTT domain): [groups][beta][l + 1 +
// n_p][N], every digit lifted to Q_l u P in the NTT domain (pool buffer, the
// caller frees it)
u64* op_modup_rows(Context& c, const Rows& d, int level);
// ModDown of one polynomial over Q_l u P (rows q_0..q_l, p_0..), NTT domain,
// into out (rows q_0..q_l)
void op_mod_down_rows(Context& c, const u64* in, int level, u64* out);
void key_switch(Context& c, const Rows& d, int level, const u64* key, u64* out0, u64* out1,
                size_t out_gstride, const Rows* add0, const Rows* add1);

}  // namespace hs
