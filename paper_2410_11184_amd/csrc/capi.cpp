// extern "C" entry points: argument checks, error capture, handle wrapping.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/hs.h"
#include "host.h"
#include "poly.h"
#include "softmax.h"
#include <chrono>
#include <memory>
#include <vector>

struct hs_ctx {
    hs::Context* c;
    double last_stats[4] = {0, 0, 0, 0};
};
struct hs_ct {
    hs::Context* c;
    hs::Ct ct;
};

static thread_local std::string g_err;

template <class F>
static hs_status guard(F&& f) {
    try {
        f();
        return HS_OK;
    } catch (const hs::Error& e) {
        g_err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        g_err = e.what();
        return HS_E_DEVICE;
    }
}

static hs_ct* wrap(hs::Context* c, const hs::Ct& ct) {
    hs_ct* h = new hs_ct;
    h->c = c;
    h->ct = ct;
    return h;
}

#define NEED(x) HS_REQUIRE((x), hs::E_ARG, "null argument: " #x)

static void check_ev(hipError_t e) { HS_REQUIRE(e == hipSuccess, hs::E_DEVICE, "hipEventCreate failed"); }

extern "C" {

const char* hs_version(void) { return "hs 0.1 (gfx950)"; }
const char* hs_last_error(void) { return g_err.c_str(); }

hs_status hs_ctx_create_ex(const hs_params* p, int device, void* stream, hs_alloc_fn alloc_fn, hs_free_fn free_fn,
                            void* user, hs_ctx** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(p);
        NEED(out);
        HS_REQUIRE((alloc_fn == nullptr) == (free_fn == nullptr), hs::E_ARG,
                   "give both allocator callbacks or neither");
        NEED(p->q_bits);
        NEED(p->p_bits);
        hs::Params q;
        q.logN = p->log_n;
        q.q_bits.assign(p->q_bits, p->q_bits + p->n_q);
        q.p_bits.assign(p->p_bits, p->p_bits + p->n_p);
        q.digit = p->digit;
        q.hamming = p->hamming;
        q.sigma = p->sigma;
        q.log_scale = p->log_scale;
        q.user_top = p->user_top;
        q.boot.cts_levels = p->boot_cts_levels;
        q.boot.evalmod_levels = p->boot_evalmod_levels;
        q.boot.stc_levels = p->boot_stc_levels;
        q.boot.K = p->boot_K;
        q.boot.double_angle = p->boot_double_angle;
        q.boot.cos_degree = p->boot_cos_degree;
        q.boot.log_boot_scale = p->boot_log_scale;
        if (q.boot.cts_levels > 0) {
            const int nb = q.boot.cts_levels + q.boot.evalmod_levels + q.boot.stc_levels;
            HS_REQUIRE(q.user_top == p->n_q - 1 - nb, hs::E_PARAM, "user_top inconsistent with bootstrapping levels");
        }
        hs::DevAllocator da;
        da.alloc_fn = alloc_fn;
        da.free_fn = free_fn;
        da.user = user;
        hs_ctx* h = new hs_ctx;
        try {
            h->c = new hs::Context(q, device, stream, &da);
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
}

hs_status hs_ctx_clone(hs_ctx* src, void* stream, hs_ctx** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(src);
        NEED(out);
        hs_ctx* h = new hs_ctx;
        try {
            h->c = new hs::Context(*src->c, stream);
        } catch (...) {
            delete h;
            throw;
        }
        *out = h;
    });
}

hs_status hs_ctx_create(const hs_params* p, int device, void* stream, hs_ctx** out) {
    return hs_ctx_create_ex(p, device, stream, nullptr, nullptr, nullptr, out);
}

void hs_ctx_destroy(hs_ctx* ctx) {
    if (!ctx) return;
    hs::destroy_context(ctx->c);
    delete ctx;
}

hs_status hs_ctx_get_info(const hs_ctx* ctx, hs_ctx_info* info) {
    return guard([&] {
        NEED(ctx);
        NEED(info);
        const hs::Context& c = *ctx->c;
        info->log_n = c.logN;
        info->n = c.N;
        info->slots = c.N / 2;
        info->n_q = c.nq;
        info->n_p = c.np;
        info->top_level = c.L;
        info->user_top = c.prm.user_top;
        info->dnum = c.dnum;
        info->digit = c.prm.digit;
        info->has_boot = c.prm.boot.cts_levels > 0;
    });
}

hs_status hs_stream_create(int device, void** stream) {
    return guard([&] {
        NEED(stream);
        *stream = nullptr;
        HS_REQUIRE(hipSetDevice(device) == hipSuccess, hs::E_DEVICE, "hipSetDevice failed");
        hipStream_t st = nullptr;
        HS_REQUIRE(hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess, hs::E_DEVICE,
                   "hipStreamCreate failed");
        *stream = (void*)st;
    });
}

hs_status hs_stream_destroy(void* stream) {
    return guard([&] {
        NEED(stream);
        HS_REQUIRE(hipStreamDestroy((hipStream_t)stream) == hipSuccess, hs::E_DEVICE, "hipStreamDestroy failed");
    });
}

hs_status hs_ctx_memory(const hs_ctx* ctx, size_t* in_use, size_t* reserved) {
    return guard([&] {
        NEED(ctx);
        if (in_use) *in_use = ctx->c->pool.bytes_in_use();
        if (reserved) *reserved = ctx->c->pool.bytes_reserved();
    });
}

hs_status hs_ctx_trim(hs_ctx* ctx, size_t* released) {
    return guard([&] {
        NEED(ctx);
        ctx->c->sync();
        const size_t r = ctx->c->pool.trim(~(size_t)0);
        if (released) *released = r;
    });
}

hs_status hs_ctx_primes(const hs_ctx* ctx, uint64_t* out, size_t cap, size_t* n) {
    return guard([&] {
        NEED(ctx);
        const auto& pr = ctx->c->primes;
        if (n) *n = pr.size();
        for (size_t i = 0; i < pr.size() && i < cap && out; i++) out[i] = pr[i];
    });
}

hs_status hs_sync(hs_ctx* ctx) {
    return guard([&] {
        NEED(ctx);
        ctx->c->sync();
    });
}

hs_status hs_keygen(hs_ctx* ctx, uint64_t seed) {
    return guard([&] {
        NEED(ctx);
        HS_REQUIRE(ctx->c->live_plans == 0, hs::E_STATE,
                   "keygen: captured Softmax schedules hold the current keys; destroy them first");
        hs::keygen(*ctx->c, seed);
    });
}

hs_status hs_add_rotation_keys(hs_ctx* ctx, const int32_t* steps, size_t n, int conj) {
    return guard([&] {
        NEED(ctx);
        HS_REQUIRE(n == 0 || steps, hs::E_ARG, "null steps");
        hs::Context& c = *ctx->c;
        for (size_t i = 0; i < n; i++) {
            const int r = ((steps[i] % (c.N / 2)) + c.N / 2) % (c.N / 2);
            if (r) hs::add_galois_key(c, hs::galois_rot(r, c.N));
        }
        if (conj) hs::add_galois_key(c, 2 * c.N - 1);
    });
}

hs_status hs_key_export(hs_ctx* ctx, int key_id, uint64_t* out, size_t cap, size_t* used) {
    return guard([&] {
        NEED(ctx);
        hs::Context& c = *ctx->c;
        HS_REQUIRE(hs::has_key(c, key_id), hs::E_KEY, "no such key");
        const size_t w = (size_t)c.dnum * 2 * (c.nq + c.np) * c.N;
        if (used) *used = w;
        if (!out || cap == 0) return;
        HS_REQUIRE(cap >= w, hs::E_ARG, "buffer too small");
        c.download(out, c.keys.at(key_id), w * 8);
        // the device copy holds the Q rows times P^-1 mod q_i: restore them
        const size_t rw = (size_t)(c.nq + c.np) * c.N;
        for (int blk = 0; blk < 2 * c.dnum; blk++)
            for (int i = 0; i < c.nq; i++) {
                const uint64_t q = c.primes[i], pm = c.P_mod[i];
                uint64_t* row = out + blk * rw + (size_t)i * c.N;
                for (int x = 0; x < c.N; x++) row[x] = hs::mulmod_h(row[x], pm, q);
            }
    });
}

hs_status hs_secret_export(hs_ctx* ctx, int64_t* out, size_t n) {
    return guard([&] {
        NEED(ctx);
        NEED(out);
        hs::Context& c = *ctx->c;
        HS_REQUIRE(c.have_keys, hs::E_STATE, "keygen first");
        HS_REQUIRE(n >= (size_t)c.N, hs::E_ARG, "buffer too small");
        std::memcpy(out, c.s_coeff.data(), sizeof(int64_t) * c.N);
    });
}

hs_status hs_pk_export(hs_ctx* ctx, uint64_t* out, size_t cap, size_t* used) {
    return guard([&] {
        NEED(ctx);
        hs::Context& c = *ctx->c;
        HS_REQUIRE(c.have_keys, hs::E_STATE, "keygen first");
        const size_t w = 2 * (size_t)c.nq * c.N;
        if (used) *used = w;
        if (!out || cap == 0) return;
        HS_REQUIRE(cap >= w, hs::E_ARG, "buffer too small");
        c.download(out, c.pk, w * 8);
    });
}

hs_status hs_encode(hs_ctx* ctx, const double* re, const double* im, size_t n_slots, int level, double scale,
                    uint64_t* out) {
    return guard([&] {
        NEED(ctx);
        NEED(re);
        NEED(out);
        hs::Context& c = *ctx->c;
        HS_REQUIRE(n_slots == (size_t)c.N / 2, hs::E_ARG, "n_slots must be N/2");
        HS_REQUIRE(level >= 0 && level <= c.L, hs::E_LEVEL, "level out of range");
        const size_t w = (size_t)(level + 1) * c.N;
        u64* d = c.alloc_words(w);
        hs::encode_to(c, d, re, im, level, scale);
        c.download(out, d, w * 8);
        c.free_words(d);
    });
}

hs_status hs_encode_encrypt(hs_ctx* ctx, const double* re, const double* im, size_t n_slots, int level,
                            double scale, uint64_t seed, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(re);
        NEED(out);
        hs::Context& c = *ctx->c;
        HS_REQUIRE(n_slots == (size_t)c.N / 2, hs::E_ARG, "n_slots must be N/2");
        HS_REQUIRE(level >= 0 && level <= c.L, hs::E_LEVEL, "level out of range");
        const size_t w = (size_t)(level + 1) * c.N;
        u64* d = c.alloc_words(w);
        hs::encode_to(c, d, re, im, level, scale);
        hs::Ct ct = hs::encrypt(c, d, level, scale, seed);
        c.free_words(d);
        *out = wrap(&c, ct);
    });
}

hs_status hs_encrypt_rows(hs_ctx* ctx, const uint64_t* pt, int level, double scale, uint64_t seed, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(pt);
        NEED(out);
        hs::Context& c = *ctx->c;
        HS_REQUIRE(level >= 0 && level <= c.L, hs::E_LEVEL, "level out of range");
        const size_t w = (size_t)(level + 1) * c.N;
        u64* d = c.alloc_words(w);
        c.upload(d, pt, w * 8);
        hs::Ct ct = hs::encrypt(c, d, level, scale, seed);
        c.free_words(d);
        *out = wrap(&c, ct);
    });
}

hs_status hs_decrypt_decode(hs_ctx* ctx, const hs_ct* ct, double* re, double* im, size_t n_slots) {
    return guard([&] {
        NEED(ctx);
        NEED(ct);
        NEED(re);
        hs::Context& c = *ctx->c;
        HS_REQUIRE(n_slots == (size_t)c.N / 2, hs::E_ARG, "n_slots must be N/2");
        hs::decrypt_decode(c, ct->ct, 0, re, im);
    });
}

hs_status hs_ct_export(hs_ctx* ctx, const hs_ct* ct, uint64_t* words, size_t cap, size_t* used) {
    return guard([&] {
        NEED(ctx);
        NEED(ct);
        hs::Context& c = *ctx->c;
        const size_t w = ct->ct.ct_words(c.N);
        if (used) *used = w;
        if (!words || cap == 0) return;
        HS_REQUIRE(cap >= w, hs::E_ARG, "buffer too small");
        c.download(words, ct->ct.d, w * 8);
    });
}

hs_status hs_ct_import(hs_ctx* ctx, const uint64_t* words, int level, int ncomp, double scale, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(words);
        NEED(out);
        hs::Context& c = *ctx->c;
        HS_REQUIRE(ncomp == 2 || ncomp == 3, hs::E_ARG, "ncomp must be 2 or 3");
        hs::Ct ct = hs::ct_alloc(c, 1, ncomp, level);
        ct.scale = scale;
        c.upload(ct.d, words, ct.ct_words(c.N) * 8);
        *out = wrap(&c, ct);
    });
}

hs_status hs_ct_info(const hs_ct* ct, int* level, int* ncomp, double* scale) {
    return guard([&] {
        NEED(ct);
        if (level) *level = ct->ct.level;
        if (ncomp) *ncomp = ct->ct.ncomp;
        if (scale) *scale = ct->ct.scale;
    });
}

hs_status hs_ct_set_scale(hs_ct* ct, double scale) {
    return guard([&] {
        NEED(ct);
        HS_REQUIRE(scale > 0, hs::E_ARG, "scale must be positive");
        ct->ct.scale = scale;
    });
}

void hs_ct_destroy(hs_ct* ct) {
    if (!ct) return;
    if (ct->c && ct->ct.d) ct->c->free_words(ct->ct.d);
    delete ct;
}

#define UNARY_OP(name, expr)                                     \
    hs_status name(hs_ctx* ctx, const hs_ct* a, hs_ct** out) {   \
        if (out) *out = nullptr;                                 \
        return guard([&] {                                       \
            NEED(ctx);                                           \
            NEED(a);                                             \
            NEED(out);                                           \
            hs::Context& c = *ctx->c;                            \
            hs::Ct r = (expr);                                   \
            *out = wrap(&c, r);                                  \
        });                                                      \
    }

hs_status hs_add(hs_ctx* ctx, const hs_ct* a, const hs_ct* b, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(b);
        NEED(out);
        *out = wrap(ctx->c, hs::op_add(*ctx->c, a->ct, b->ct));
    });
}

hs_status hs_sub(hs_ctx* ctx, const hs_ct* a, const hs_ct* b, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(b);
        NEED(out);
        *out = wrap(ctx->c, hs::op_sub(*ctx->c, a->ct, b->ct));
    });
}

hs_status hs_tensor(hs_ctx* ctx, const hs_ct* a, const hs_ct* b, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(b);
        NEED(out);
        *out = wrap(ctx->c, hs::op_tensor(*ctx->c, a->ct, b->ct));
    });
}

UNARY_OP(hs_relinearize, hs::op_relin(c, a->ct))

hs_status hs_rescale(hs_ctx* ctx, const hs_ct* a, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(out);
        *out = wrap(ctx->c, hs::op_rescale(*ctx->c, a->ct));
    });
}

hs_status hs_mult_relin(hs_ctx* ctx, const hs_ct* a, const hs_ct* b, int rescale, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(b);
        NEED(out);
        hs::Context& c = *ctx->c;
        if (rescale) {
            *out = wrap(&c, hs::op_mult(c, a->ct, b->ct));
        } else {
            hs::Ct d = hs::op_tensor(c, a->ct, b->ct);
            hs::Ct r = hs::op_relin(c, d);
            hs::ct_free(c, d);
            *out = wrap(&c, r);
        }
    });
}

// Scratch bytes of op_mult_into at one level (one ciphertext), by the order of
// its allocations: tensor d, relinearised r (rescale only), ModUp's extension
// and coefficient copy, then the inner product and the conversion; the
// rescale's two buffers fit in the tensor's freed block.
static size_t mult_scratch_bytes(const hs::Context& c, int level, bool rescale) {
    const size_t row = (size_t)c.N * 8;
    auto blk = [&](size_t rows) { return (rows * row + 255) & ~(size_t)255; };
    const size_t nql = (size_t)level + 1, E = nql + c.np;
    const size_t beta = (nql + c.prm.digit - 1) / c.prm.digit;
    const size_t base = blk(3 * nql) + (rescale ? blk(2 * nql) : 0) + blk(beta * E);
    return std::max(base + blk(nql), base + blk(2 * E) + blk(2 * nql));
}

hs_status hs_mult_relin_noalloc(hs_ctx* ctx, const uint64_t* a, const uint64_t* b, int level, double scale_a,
                                double scale_b, int rescale, uint64_t* out, double* out_scale) {
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(b);
        NEED(out);
        hs::Context& c = *ctx->c;
        HS_REQUIRE(level >= 0 && level <= c.L, hs::E_LEVEL, "level out of range");
        HS_REQUIRE(!rescale || level >= 1, hs::E_LEVEL, "rescale needs level >= 1");
        HS_REQUIRE(scale_a > 0 && scale_b > 0, hs::E_ARG, "scales must be positive");
        const size_t need = mult_scratch_bytes(c, level, rescale != 0);
        if (need > hs::kScratchBytes) {
            char msg[200];
            std::snprintf(msg, sizeof msg, "this level needs %.1f MiB of scratch; the fixed scratch holds %.0f MiB",
                          need / 1048576.0, hs::kScratchBytes / 1048576.0);
            throw hs::Error(hs::E_ARG, msg);
        }
        const size_t in_bytes = (size_t)2 * (level + 1) * c.N * 8;
        const size_t out_bytes = (size_t)2 * (level + (rescale ? 0 : 1)) * c.N * 8;
        for (const void* p : {(const void*)a, (const void*)b, (const void*)out})
            HS_REQUIRE(((uintptr_t)p & 255) == 0, hs::E_ARG, "device pointers must be 256-byte aligned");
        auto overlap = [](const void* x, size_t nx, const void* y, size_t ny) {
            const uintptr_t u = (uintptr_t)x, v = (uintptr_t)y;
            return u < v + ny && v < u + nx;
        };
        HS_REQUIRE(!overlap(out, out_bytes, a, in_bytes) && !overlap(out, out_bytes, b, in_bytes), hs::E_ARG,
                   "out overlaps an input");
        HS_REQUIRE(hs::has_key(c, 0), hs::E_KEY, "relinearisation key missing");
        HS_REQUIRE(!hs::prof_enabled(c.T.prof), hs::E_STATE, "the launch profiler allocates events: disable it");
        const int nql = level + 1;
        const int beta = (nql + c.prm.digit - 1) / c.prm.digit;
        for (int j = 0; j < beta; j++)
            HS_REQUIRE(c.modup.count(std::make_pair(level, j)) != 0, hs::E_STATE,
                       "key-switching tables of this level not built yet: run one hs_mult_relin at this level first");
        HS_REQUIRE(c.moddown.count(level) != 0, hs::E_STATE,
                   "key-switching tables of this level not built yet: run one hs_mult_relin at this level first");
        void* base = hs::scratch_device_ptr(c.device);
        HS_REQUIRE(base != nullptr, hs::E_DEVICE, "device address of the scratch array unknown (lookup failed)");
        hs::Pool sp;
        sp.adopt(base, hs::kScratchBytes);
        hs::Pool* prev = c.cur;
        c.cur = &sp;
        hs::tune_suspend(true);
        struct Restore {
            hs::Context& c;
            hs::Pool* prev;
            ~Restore() {
                c.cur = prev;
                hs::tune_suspend(false);
            }
        } restore{c, prev};
        hs::Ct A, B;
        A.d = const_cast<uint64_t*>(a);
        B.d = const_cast<uint64_t*>(b);
        A.level = B.level = level;
        A.scale = scale_a;
        B.scale = scale_b;
        const double s = hs::op_mult_into(c, A, B, rescale != 0, out);
        if (out_scale) *out_scale = s;
    });
}

hs_status hs_rotate(hs_ctx* ctx, const hs_ct* a, int32_t r, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(out);
        *out = wrap(ctx->c, hs::op_rotate(*ctx->c, a->ct, r));
    });
}

hs_status hs_rotate_hoisted(hs_ctx* ctx, const hs_ct* a, const int32_t* rots, size_t n, hs_ct** out) {
    if (out)
        for (size_t i = 0; i < n; i++) out[i] = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(rots);
        NEED(out);
        HS_REQUIRE(n >= 1 && n <= (size_t)hs::kMaxKeys, hs::E_ARG, "1 to 32 rotations");
        hs::Context& c = *ctx->c;
        const std::vector<int> rs(rots, rots + n);
        hs::Ct b = hs::op_rotate_hoisted_batch(c, a->ct, rs);
        for (size_t i = 0; i < n; i++) out[i] = wrap(&c, hs::ct_slice(c, b, (int)(i * a->ct.m), a->ct.m));
        hs::ct_free(c, b);
    });
}

hs_status hs_rotate_batch(hs_ctx* ctx, const hs_ct* const* a, const int32_t* rots, size_t n, hs_ct** out) {
    if (out)
        for (size_t i = 0; i < n; i++) out[i] = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(rots);
        NEED(out);
        HS_REQUIRE(n >= 1 && n <= (size_t)hs::kMaxKeys, hs::E_ARG, "1 to 32 ciphertexts");
        hs::Context& c = *ctx->c;
        std::vector<const hs::Ct*> parts;
        std::vector<int> gal;
        const int half = c.N / 2;
        for (size_t i = 0; i < n; i++) {
            NEED(a[i]);
            HS_REQUIRE(a[i]->ct.m == 1, hs::E_ARG, "one ciphertext per handle");
            HS_REQUIRE(a[i]->ct.scale == a[0]->ct.scale, hs::E_SCALE, "inputs must share one scale");
            HS_REQUIRE(((rots[i] % half) + half) % half != 0, hs::E_ARG, "zero rotation");
            parts.push_back(&a[i]->ct);
            gal.push_back(hs::galois_rot(rots[i], c.N));
        }
        hs::Ct in = hs::ct_gather(c, parts);   // checks the levels
        hs::Ct b;
        try {
            b = hs::op_galois_batch(c, in, gal, 1);
        } catch (...) {
            hs::ct_free(c, in);
            throw;
        }
        hs::ct_free(c, in);
        for (size_t i = 0; i < n; i++) out[i] = wrap(&c, hs::ct_slice(c, b, (int)i, 1));
        hs::ct_free(c, b);
    });
}

UNARY_OP(hs_conjugate, hs::op_conjugate(c, a->ct))

hs_status hs_mul_plain_rows(hs_ctx* ctx, const hs_ct* a, const uint64_t* pt, double pt_scale, int rescale,
                            hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(pt);
        NEED(out);
        hs::Context& c = *ctx->c;
        const size_t w = (size_t)(a->ct.level + 1) * c.N;
        u64* d = c.alloc_words(w);
        c.upload(d, pt, w * 8);
        hs::Ct r = hs::op_mul_plain(c, a->ct, d, pt_scale, rescale != 0);
        c.sync();
        c.free_words(d);
        *out = wrap(&c, r);
    });
}

hs_status hs_mul_int(hs_ctx* ctx, const hs_ct* a, int64_t k, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(out);
        hs::Context& c = *ctx->c;
        hs::Ct r = hs::ct_copy(c, a->ct);
        hs::op_mul_int_inplace(c, r, (long long)k);
        *out = wrap(&c, r);
    });
}

hs_status hs_add_const(hs_ctx* ctx, const hs_ct* a, double v, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(out);
        hs::Context& c = *ctx->c;
        hs::Ct r = hs::ct_copy(c, a->ct);
        hs::op_add_const_inplace(c, r, v);
        *out = wrap(&c, r);
    });
}

hs_status hs_mod_drop(hs_ctx* ctx, const hs_ct* a, int level, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(out);
        *out = wrap(ctx->c, hs::ct_drop(*ctx->c, a->ct, level));
    });
}

hs_status hs_mod_raise(hs_ctx* ctx, const hs_ct* a, int level, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(out);
        *out = wrap(ctx->c, hs::op_mod_raise(*ctx->c, a->ct, level));
    });
}

hs_status hs_mul_monomial(hs_ctx* ctx, const hs_ct* a, int k, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(out);
        *out = wrap(ctx->c, hs::op_mul_monomial(*ctx->c, a->ct, k));
    });
}

hs_status hs_dbg_minimax(double a, double b, int degree, double e, double* c) {
    return guard([&] {
        NEED(c);
        const hs::ChebPoly p = hs::minimax_invpow(a, b, degree, e);
        for (int j = 0; j <= degree; j++) c[j] = p.c[j];
    });
}

hs_status hs_dbg_mul_rate(hs_ctx* ctx, double* tops) {
    return guard([&] {
        NEED(ctx);
        NEED(tops);
        *tops = hs::k_mul_rate(ctx->c->stream);
        HS_REQUIRE(*tops > 0, hs::E_DEVICE, "multiplier probe failed");
    });
}

hs_status hs_dbg_ntt_time(hs_ctx* ctx, int groups, int level, int reps, int inverse, double* us) {
    return guard([&] {
        NEED(ctx);
        NEED(us);
        hs::Context& c = *ctx->c;
        HS_REQUIRE(level >= 0 && level <= c.L, hs::E_LEVEL, "level out of range");
        HS_REQUIRE(groups >= 1 && groups <= 4096 && reps >= 1 && reps <= 1000, hs::E_ARG, "groups or reps");
        HS_REQUIRE(!c.capturing, hs::E_STATE, "not while capturing");
        const int rpg = level + 1;
        const size_t w = (size_t)groups * rpg * c.N;
        u64* d = c.alloc_words(w);
        hs::Rows r{d, groups, rpg, (size_t)rpg * c.N, rpg, 0, c.nq};
        hs::k_sample_uniform(c.T, r, 0x5eedull, 0x7000000000000000ull, c.stream);
        hs::k_ntt(c.T, r, inverse != 0, c.stream);                    // warm
        hipEvent_t e0, e1;
        check_ev(hipEventCreate(&e0));
        check_ev(hipEventCreate(&e1));
        (void)hipEventRecord(e0, (hipStream_t)c.stream);
        for (int i = 0; i < reps; i++) hs::k_ntt(c.T, r, inverse != 0, c.stream);
        (void)hipEventRecord(e1, (hipStream_t)c.stream);
        (void)hipEventSynchronize(e1);
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        c.free_words(d);
        *us = 1e3 * ms / reps;
    });
}

hs_status hs_dbg_ntt(hs_ctx* ctx, int prime, uint64_t* rows, size_t nrows, int inverse) {
    return guard([&] {
        NEED(ctx);
        NEED(rows);
        hs::Context& c = *ctx->c;
        HS_REQUIRE(prime >= 0 && prime < c.nq + c.np, hs::E_ARG, "prime index out of range");
        const size_t w = nrows * c.N;
        u64* d = c.alloc_words(w);
        c.upload(d, rows, w * 8);
        hs::Rows r{d, (int)nrows, 1, (size_t)c.N, 1, prime, c.nq};
        if (prime >= c.nq) {
            r.nq = 0;
            r.p_base = prime;
        }
        hs::k_ntt(c.T, r, inverse != 0, c.stream);
        c.download(rows, d, w * 8);
        c.free_words(d);
    });
}

hs_status hs_dbg_ring(hs_ctx* ctx, int op, int level, int arg, const uint64_t* in, size_t in_words, uint64_t* out,
                      size_t out_cap, size_t* out_words) {
    return guard([&] {
        NEED(ctx);
        NEED(in);
        hs::Context& c = *ctx->c;
        HS_REQUIRE(level >= 0 && level <= c.L, hs::E_LEVEL, "level out of range");
        const size_t N = c.N, nql = (size_t)level + 1, E = nql + c.np;
        const size_t beta = (nql + c.prm.digit - 1) / c.prm.digit;
        size_t win = nql * N, wout = nql * N;
        switch (op) {
            case HS_DBG_NTT:
            case HS_DBG_INTT:
            case HS_DBG_AUTO: break;
            case HS_DBG_MODUP: wout = beta * E * N; break;
            case HS_DBG_MODDOWN: win = E * N; break;
            case HS_DBG_RESCALE:
                HS_REQUIRE(level >= 1, hs::E_LEVEL, "rescale needs level >= 1");
                wout = (nql - 1) * N;
                break;
            case HS_DBG_TENSOR:
                win = 4 * nql * N;
                wout = 3 * nql * N;
                break;
            default: throw hs::Error(hs::E_ARG, "unknown ring operation");
        }
        if (out_words) *out_words = wout;
        HS_REQUIRE(in_words == win, hs::E_ARG, "input size does not match the operation and level");
        if (!out || out_cap == 0) return;
        HS_REQUIRE(out_cap >= wout, hs::E_ARG, "output buffer too small");
        u64* din = c.alloc_words(win);
        c.upload(din, in, win * 8);
        u64* dout = nullptr;
        hs::Ct tmp;
        switch (op) {
            case HS_DBG_NTT:
            case HS_DBG_INTT: {
                dout = c.alloc_words(wout);
                hs::Rows rs = c.rows(din, 1, (int)nql, win), rd = c.rows(dout, 1, (int)nql, wout);
                hs::k_ntt_from(c.T, rd, rs, op == HS_DBG_INTT, c.stream);
                break;
            }
            case HS_DBG_MODUP:
                dout = hs::op_modup_rows(c, c.rows(din, 1, (int)nql, win), level);
                break;
            case HS_DBG_MODDOWN:
                dout = c.alloc_words(wout);
                hs::op_mod_down_rows(c, din, level, dout);
                break;
            case HS_DBG_AUTO: {
                HS_REQUIRE(arg % 2 != 0, hs::E_ARG, "the Galois element must be odd");
                const int g = ((arg % (2 * c.N)) + 2 * c.N) % (2 * c.N);
                dout = c.alloc_words(wout);
                hs::k_permute(c.T, c.rows(dout, 1, (int)nql, wout), c.rows(din, 1, (int)nql, win), c.perm(g),
                              c.stream);
                break;
            }
            case HS_DBG_RESCALE: {
                hs::Ct a;
                a.d = din;
                a.m = 1;
                a.ncomp = 1;
                a.level = level;
                tmp = hs::op_rescale(c, a);
                dout = tmp.d;
                break;
            }
            case HS_DBG_TENSOR: {
                hs::Ct a, b;
                a.d = din;
                a.level = b.level = level;
                b.d = din + 2 * nql * N;
                tmp = hs::op_tensor(c, a, b);
                dout = tmp.d;
                break;
            }
        }
        c.download(out, dout, wout * 8);
        c.free_words(din);
        c.free_words(dout);
    });
}

static hs::SoftmaxOpts softmax_opts(const hs_softmax_opts* opts) {
    hs::SoftmaxOpts o;
    if (opts) {
        o.variant = opts->variant;
        o.k = opts->k;
        if (opts->exp_degree > 0) o.exp_degree = opts->exp_degree;
        if (opts->inv_degree_first > 0) o.inv_degree_first = opts->inv_degree_first;
        if (opts->inv_degree_mid > 0) o.inv_degree_mid = opts->inv_degree_mid;
        if (opts->inv_degree_last > 0) o.inv_degree_last = opts->inv_degree_last;
        o.debug_stop = opts->debug_stop;
        if (opts->power > 0) o.power = opts->power;
        o.newton_steps = opts->newton_steps;
        o.mask_mode = opts->mask_mode;
        o.approx = opts->approx;
        o.merge = opts->merge;
    }
    return o;
}

static hs_status softmax_impl(hs_ctx* ctx, hs_ct* const* in, size_t m, size_t njobs, uint32_t n, double M,
                              const hs_softmax_opts* opts, hs_ct** out) {
    if (out)
        for (size_t i = 0; i < m; i++) out[i] = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(in);
        NEED(out);
        HS_REQUIRE(m >= 1, hs::E_ARG, "m must be >= 1");
        HS_REQUIRE(njobs >= 1 && m % njobs == 0, hs::E_ARG, "the ciphertext count must be a multiple of the job count");
        hs::Context& c = *ctx->c;
        std::vector<const hs::Ct*> parts;
        for (size_t i = 0; i < m; i++) {
            HS_REQUIRE(in[i] != nullptr, hs::E_ARG, "null input ciphertext");
            HS_REQUIRE(in[i]->ct.scale == in[0]->ct.scale, hs::E_SCALE, "inputs must share one scale");
            parts.push_back(&in[i]->ct);
        }
        const hs::SoftmaxOpts o = softmax_opts(opts);
        auto t0 = std::chrono::steady_clock::now();
        hs::Ct batch = hs::ct_gather(c, parts);
        hs::SoftmaxStats st;
        hs::Ct y;
        try {
            y = hs::softmax(c, batch, (int)n, M, o, &st, (int)njobs);
        } catch (...) {
            hs::ct_free(c, batch);
            throw;
        }
        hs::ct_free(c, batch);
        for (size_t i = 0; i < m; i++) out[i] = wrap(&c, hs::ct_slice(c, y, (int)i, 1));
        hs::ct_free(c, y);
        c.sync();
        auto t1 = std::chrono::steady_clock::now();
        ctx->last_stats[0] = st.k;
        ctx->last_stats[1] = st.bootstraps;
        ctx->last_stats[2] = st.levels_left;
        ctx->last_stats[3] = std::chrono::duration<double, std::milli>(t1 - t0).count();
    });
}

hs_status hs_softmax(hs_ctx* ctx, hs_ct* const* in, size_t m, uint32_t n, double M, const hs_softmax_opts* opts,
                     hs_ct** out) {
    return softmax_impl(ctx, in, m, 1, n, M, opts, out);
}

hs_status hs_softmax_jobs(hs_ctx* ctx, hs_ct* const* in, size_t m, size_t njobs, uint32_t n, double M,
                          const hs_softmax_opts* opts, hs_ct** out) {
    return softmax_impl(ctx, in, m, njobs, n, M, opts, out);
}

// ------------------------------------------------- captured Softmax schedules
// The schedule of one Softmax call (fixed ciphertext count, job count,
// dimension, range, options, input level and scale) recorded once as a HIP
// graph.  The plan owns a private arena: the graph's intermediate buffers keep
// their addresses for every replay, so no other allocation may ever get them.
struct hs_softmax_plan {
    hs_ctx* ctx = nullptr;
    hs::Pool pool;
    hipStream_t stream = nullptr;   // capture and replay stream (a context may run on the null stream)
    hs::Ct in, out;
    int level = 0, ncomp = 2;
    double scale = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double stats[3] = {0, 0, 0};
    bool counted = false;           // included in the context's live_plans
    ~hs_softmax_plan() {
        if (counted) ctx->c->live_plans--;
        if (stream) (void)hipStreamSynchronize(stream);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        pool.release_all();
        if (stream) (void)hipStreamDestroy(stream);
    }
};

namespace {
// Points the context at the plan's arena and stream for the lifetime of the scope.
struct PlanScope {
    hs::Context& c;
    void* stream0;
    PlanScope(hs::Context& cc, hs_softmax_plan& p) : c(cc), stream0(cc.stream) {
        c.cur = &p.pool;
        c.stream = p.stream;
    }
    ~PlanScope() {
        c.capturing = false;
        c.cur = &c.pool;
        c.stream = stream0;
    }
};
}  // namespace

hs_status hs_softmax_plan_create(hs_ctx* ctx, hs_ct* const* in, size_t m, size_t njobs, uint32_t n, double M,
                                 const hs_softmax_opts* opts, hs_softmax_plan** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(in);
        NEED(out);
        HS_REQUIRE(m >= 1, hs::E_ARG, "m must be >= 1");
        HS_REQUIRE(njobs >= 1 && m % njobs == 0, hs::E_ARG, "the ciphertext count must be a multiple of the job count");
        hs::Context& c = *ctx->c;
        HS_REQUIRE(!c.capturing && c.cur == &c.pool, hs::E_STATE, "a schedule is already being captured");
        HS_REQUIRE(!hs::prof_enabled(c.T.prof), hs::E_STATE, "disable the launch profiler before capturing");
        std::vector<const hs::Ct*> parts;
        for (size_t i = 0; i < m; i++) {
            HS_REQUIRE(in[i] != nullptr, hs::E_ARG, "null input ciphertext");
            HS_REQUIRE(in[i]->ct.m == 1, hs::E_ARG, "one ciphertext per handle");
            HS_REQUIRE(in[i]->ct.scale == in[0]->ct.scale, hs::E_SCALE, "inputs must share one scale");
            parts.push_back(&in[i]->ct);
        }
        const hs::SoftmaxOpts o = softmax_opts(opts);
        std::unique_ptr<hs_softmax_plan> P(new hs_softmax_plan);
        P->ctx = ctx;
        P->pool.set_source(&ctx->c->da);   // the plan's arena draws on the context's allocator
        HS_REQUIRE(hipStreamCreateWithFlags(&P->stream, hipStreamNonBlocking) == hipSuccess, hs::E_DEVICE,
                   "hipStreamCreate failed");
        c.sync();                                   // inputs were produced on the context's stream
        PlanScope scope(c, *P);
        P->in = hs::ct_gather(c, parts);            // the plan's input buffer
        P->level = P->in.level;
        P->ncomp = P->in.ncomp;
        P->scale = P->in.scale;
        {
            // eager run: builds every table and key the schedule touches and
            // sizes the plan's arena, so the recording needs no host work
            hs::SoftmaxStats st;
            hs::Ct y = hs::softmax(c, P->in, (int)n, M, o, &st, (int)njobs);
            hs::ct_free(c, y);
            c.sync();
        }
        HS_REQUIRE(hipStreamBeginCapture(P->stream, hipStreamCaptureModeRelaxed) == hipSuccess, hs::E_DEVICE,
                   "hipStreamBeginCapture failed");
        c.capturing = true;
        hs::SoftmaxStats st;
        try {
            P->out = hs::softmax(c, P->in, (int)n, M, o, &st, (int)njobs);
        } catch (...) {
            c.capturing = false;
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(P->stream, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        c.capturing = false;
        HS_REQUIRE(hipStreamEndCapture(P->stream, &P->graph) == hipSuccess && P->graph, hs::E_DEVICE,
                   "hipStreamEndCapture failed");
        HS_REQUIRE(hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0) == hipSuccess, hs::E_DEVICE,
                   "hipGraphInstantiate failed");
        P->stats[0] = st.k;
        P->stats[1] = st.bootstraps;
        P->stats[2] = st.levels_left;
        c.live_plans++;
        P->counted = true;
        *out = P.release();
    });
}

hs_status hs_softmax_plan_run(hs_softmax_plan* plan, hs_ct* const* in, size_t m, hs_ct** out) {
    if (out)
        for (size_t i = 0; i < m; i++) out[i] = nullptr;
    return guard([&] {
        NEED(plan);
        NEED(in);
        NEED(out);
        hs::Context& c = *plan->ctx->c;
        HS_REQUIRE(m == (size_t)plan->in.m, hs::E_ARG, "ciphertext count differs from the plan's");
        for (size_t i = 0; i < m; i++) {
            HS_REQUIRE(in[i] != nullptr, hs::E_ARG, "null input ciphertext");
            const hs::Ct& a = in[i]->ct;
            HS_REQUIRE(a.m == 1 && a.level == plan->level && a.ncomp == plan->ncomp, hs::E_LEVEL,
                       "input level or size differs from the plan's");
            HS_REQUIRE(a.scale == plan->scale, hs::E_SCALE, "input scale differs from the plan's");
        }
        HS_REQUIRE(!c.capturing && c.cur == &c.pool, hs::E_STATE, "a schedule is being captured");
        auto t0 = std::chrono::steady_clock::now();
        c.sync();                                   // inputs were produced on the context's stream
        void* stream0 = c.stream;
        c.stream = plan->stream;
        try {
            const size_t w = plan->in.ct_words(c.N);
            for (size_t i = 0; i < m; i++) {
                hs::Rows dst = c.ct_rows(in[i]->ct);
                dst.base = plan->in.d + i * w;
                hs::k_copy_rows(c.T, dst, c.ct_rows(in[i]->ct), c.stream);
            }
            HS_REQUIRE(hipGraphLaunch(plan->exec, plan->stream) == hipSuccess, hs::E_DEVICE, "hipGraphLaunch failed");
            for (size_t i = 0; i < m; i++) out[i] = wrap(&c, hs::ct_slice(c, plan->out, (int)i, 1));
            c.sync();
        } catch (...) {
            c.stream = stream0;
            for (size_t i = 0; i < m; i++) {
                if (out[i]) hs_ct_destroy(out[i]);
                out[i] = nullptr;
            }
            throw;
        }
        c.stream = stream0;
        auto t1 = std::chrono::steady_clock::now();
        plan->ctx->last_stats[0] = plan->stats[0];
        plan->ctx->last_stats[1] = plan->stats[1];
        plan->ctx->last_stats[2] = plan->stats[2];
        plan->ctx->last_stats[3] = std::chrono::duration<double, std::milli>(t1 - t0).count();
    });
}

hs_status hs_softmax_plan_info(const hs_softmax_plan* plan, size_t* nodes, size_t* arena_bytes) {
    return guard([&] {
        NEED(plan);
        if (nodes) {
            size_t k = 0;
            HS_REQUIRE(hipGraphGetNodes(plan->graph, nullptr, &k) == hipSuccess, hs::E_DEVICE,
                       "hipGraphGetNodes failed");
            *nodes = k;
        }
        if (arena_bytes) *arena_bytes = plan->pool.bytes_reserved();
    });
}

void hs_softmax_plan_destroy(hs_softmax_plan* plan) { delete plan; }

// ------------------------------------------------------------- autotuner
hs_status hs_tune_enable(int on) {
    return guard([&] { hs::tune_enable(on != 0); });
}

hs_status hs_tune_clear(void) {
    return guard([&] { hs::tune_clear(); });
}

hs_status hs_tune_report(char* buf, size_t cap, size_t* used) {
    return guard([&] {
        NEED(used);
        const std::string s = hs::tune_dump();
        *used = s.size() + 1;
        if (buf && cap) {
            const size_t n = std::min(cap - 1, s.size());
            std::memcpy(buf, s.data(), n);
            buf[n] = 0;
        }
    });
}

hs_status hs_tune_save(const char* path) {
    return guard([&] {
        NEED(path);
        FILE* f = std::fopen(path, "w");
        HS_REQUIRE(f != nullptr, hs::E_ARG, "cannot open the tuning file for writing");
        const std::string s = hs::tune_dump();
        const size_t w = std::fwrite(s.data(), 1, s.size(), f);
        std::fclose(f);
        HS_REQUIRE(w == s.size(), hs::E_ARG, "short write of the tuning file");
    });
}

hs_status hs_tune_load(const char* path, int* entries) {
    return guard([&] {
        NEED(path);
        FILE* f = std::fopen(path, "r");
        HS_REQUIRE(f != nullptr, hs::E_ARG, "cannot open the tuning file");
        std::string s;
        char buf[4096];
        size_t r;
        while ((r = std::fread(buf, 1, sizeof(buf), f)) > 0) s.append(buf, r);
        std::fclose(f);
        const int n = hs::tune_load(s);
        if (entries) *entries = n;
    });
}

hs_status hs_op_counts(hs_ctx* ctx, double* out, size_t n, int clear) {
    return guard([&] {
        NEED(ctx);
        hs::Context& c = *ctx->c;
        const size_t total = (size_t)hs::OC_COUNT * hs::kMaxRows;
        if (out)
            for (size_t i = 0; i < std::min(n, total); i++) out[i] = c.opc[i / hs::kMaxRows][i % hs::kMaxRows];
        if (clear)
            for (int k = 0; k < hs::OC_COUNT; k++)
                for (int l = 0; l < hs::kMaxRows; l++) c.opc[k][l] = 0;
    });
}

hs_status hs_softmax_stats(hs_ctx* ctx, double* out, size_t n) {
    return guard([&] {
        NEED(ctx);
        NEED(out);
        for (size_t i = 0; i < n && i < 4; i++) out[i] = ctx->last_stats[i];
    });
}

hs_status hs_pack_softmax(const double* logits, size_t L, uint32_t n, size_t slots, double M, double* out,
                          size_t* m_out) {
    return guard([&] {
        NEED(logits);
        NEED(m_out);
        size_t np2 = 1;
        while (np2 < n) np2 <<= 1;
        HS_REQUIRE(n >= 1 && np2 <= slots, hs::E_PARAM, "n must be <= slots");
        HS_REQUIRE((L * np2) % slots == 0 && L * np2 >= slots, hs::E_ARG,
                   "L times the padded dimension must be a multiple of the slot count");
        const size_t m = L * np2 / slots;
        HS_REQUIRE(np2 % m == 0, hs::E_ARG, "m must divide the padded dimension");
        *m_out = m;
        for (size_t i = 0; i < L * n; i++)
            HS_REQUIRE(logits[i] >= -M && logits[i] <= 0.0, hs::E_RANGE, "logit outside [-M, 0]");
        if (!out) return;
        const size_t per = np2 / m;
        for (size_t j = 0; j < m; j++)
            for (size_t c = 0; c < per; c++)
                for (size_t l = 0; l < L; l++) {
                    const size_t coord = j * per + c;
                    out[j * slots + c * L + l] = coord < n ? logits[l * n + coord] : -M;
                }
    });
}

hs_status hs_unpack_softmax(const double* slots_in, size_t m, uint32_t n, size_t slots, double* out) {
    return guard([&] {
        NEED(slots_in);
        NEED(out);
        size_t np2 = 1;
        while (np2 < n) np2 <<= 1;
        HS_REQUIRE(m >= 1 && n >= 1 && np2 % m == 0 && (m * slots) % np2 == 0, hs::E_ARG, "bad shape");
        const size_t L = m * slots / np2, per = np2 / m;
        for (size_t j = 0; j < m; j++)
            for (size_t c = 0; c < per; c++) {
                const size_t coord = j * per + c;
                if (coord >= n) continue;
                for (size_t l = 0; l < L; l++) out[l * n + coord] = slots_in[j * slots + c * L + l];
            }
    });
}

hs_status hs_bootstrap(hs_ctx* ctx, const hs_ct* a, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(out);
        hs::Context& c = *ctx->c;
        HS_REQUIRE(hs::can_bootstrap(c), hs::E_PARAM, "no bootstrapping parameters");
        *out = wrap(&c, hs::bootstrap(c, a->ct, 1.0));
    });
}

hs_status hs_prof_enable(hs_ctx* ctx, int on) {
    return guard([&] {
        NEED(ctx);
        hs::prof_enable(ctx->c->T.prof, on != 0);
    });
}

hs_status hs_prof_collect(hs_ctx* ctx, double* out, size_t n) {
    return guard([&] {
        NEED(ctx);
        NEED(out);
        HS_REQUIRE(n >= 3 * (size_t)hs::PK_COUNT, hs::E_ARG, "buffer too small");
        hs::prof_collect(ctx->c->T.prof, out);
    });
}

hs_status hs_dbg_bootstrap_stage(hs_ctx* ctx, const hs_ct* a, int stage, hs_ct** out) {
    if (out) *out = nullptr;
    return guard([&] {
        NEED(ctx);
        NEED(a);
        NEED(out);
        hs::Context& c = *ctx->c;
        HS_REQUIRE(hs::can_bootstrap(c), hs::E_PARAM, "no bootstrapping parameters");
        HS_REQUIRE(stage >= 1 && stage <= 9, hs::E_ARG, "stage must be 1..9");
        *out = wrap(&c, hs::bootstrap_stage(c, a->ct, 1.0, stage));
    });
}

}  // extern "C"
