// Context set-up: primes, roots of unity, NTT and encoding twiddles, device
// tables, memory pool, base-conversion constants, key generation, encoding,
// encryption and decryption.
//
// The paper runs CKKS through an external library and specifies none of its
// internals (Section 5.1, Table "tab:fgb_data" gives only totals); the
// choices below are this library's own, stated where they are made.
#include <hip/hip_runtime_api.h>
#include <quadmath.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "host.h"

namespace hs {

void launch_error(const char* what) { throw Error(E_ARG, what); }

static void check_hip(hipError_t e, const char* what) {
    if (e != hipSuccess) throw Error(E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------- arithmetic
u64 mulmod_h(u64 a, u64 b, u64 q) { return (u64)((u128)a * b % q); }
u64 powmod_h(u64 a, u64 e, u64 q) {
    u64 r = 1 % q;
    a %= q;
    while (e) {
        if (e & 1) r = mulmod_h(r, a, q);
        a = mulmod_h(a, a, q);
        e >>= 1;
    }
    return r;
}
u64 invmod_h(u64 a, u64 q) { return powmod_h(a, q - 2, q); }
u64 shoup_h(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }
int galois_rot(int r, int N) {
    const int slots = N / 2;
    int rr = ((r % slots) + slots) % slots;
    return (int)powmod_h(5, (u64)rr, 2 * (u64)N);
}

// Deterministic Miller-Rabin for 64-bit integers (bases 2..37 suffice).
static bool is_prime(u64 n) {
    if (n < 2) return false;
    static const u64 small[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    for (u64 p : small) {
        if (n % p == 0) return n == p;
    }
    u64 d = n - 1;
    int s = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        s++;
    }
    for (u64 a : small) {
        u64 x = powmod_h(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool comp = true;
        for (int r = 1; r < s; r++) {
            x = mulmod_h(x, x, n);
            if (x == n - 1) {
                comp = false;
                break;
            }
        }
        if (comp) return false;
    }
    return true;
}

// Prime rule: for bit size b the candidates are 2^b + 1 + j 2N for
// j = 1, -1, 2, -2, ...; each chain entry takes the next unused prime of its
// size, Q primes first, then P primes.
static std::vector<u64> find_primes(int logN, const std::vector<int>& bits) {
    const u64 step = 2ull << logN;
    std::map<int, long long> cursor;
    std::vector<u64> out;
    for (int b : bits) {
        long long j = cursor[b];
        while (true) {
            long long k = j / 2 + 1;
            long long sign = (j % 2 == 0) ? 1 : -1;
            j++;
            u128 cand = ((u128)1 << b) + 1 + (u128)(sign > 0 ? k * step : 0) - (u128)(sign < 0 ? k * step : 0);
            u64 c = (u64)cand;
            if (c < 3 || std::find(out.begin(), out.end(), c) != out.end()) continue;
            if (is_prime(c)) {
                cursor[b] = j;
                out.push_back(c);
                break;
            }
        }
    }
    return out;
}

// psi: the smallest primitive 2N-th root of unity mod q.
static u64 smallest_psi(u64 q, int N) {
    const u64 M = 2 * (u64)N;
    u64 g = 0;
    for (u64 x = 2;; x++) {
        g = powmod_h(x, (q - 1) / M, q);
        if (powmod_h(g, (u64)N, q) == q - 1) break;
    }
    u64 best = g, cur = g, g2 = mulmod_h(g, g, q);
    for (int i = 0; i < N; i++) {
        if (cur < best) best = cur;
        cur = mulmod_h(cur, g2, q);
    }
    return best;
}

static u64 brv(u64 x, int bits) {
    u64 r = 0;
    for (int i = 0; i < bits; i++) {
        r = (r << 1) | (x & 1);
        x >>= 1;
    }
    return r;
}

// ----------------------------------------------------------------- pool
static constexpr size_t kChunk = (size_t)8 << 30;

void* DevAllocator::get(size_t bytes) const {
    if (alloc_fn) return alloc_fn(bytes, stream, user);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void DevAllocator::put(void* p, size_t bytes) const {
    if (!p) return;
    if (free_fn) free_fn(p, bytes, user);
    else (void)hipFree(p);
}

void* Pool::get_chunk(size_t bytes) {
    if (src_) return src_->get(bytes);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void Pool::put_chunk(void* p, size_t bytes) {
    if (src_) src_->put(p, bytes);
    else (void)hipFree(p);
}

void Pool::add_free(int c, size_t off, size_t size) {
    chunks_[c].free_[off] = size;
    by_size_.emplace(size, std::make_pair(c, off));
}

void Pool::remove_free(int c, size_t off, size_t size) {
    chunks_[c].free_.erase(off);
    auto range = by_size_.equal_range(size);
    for (auto it = range.first; it != range.second; ++it)
        if (it->second.first == c && it->second.second == off) {
            by_size_.erase(it);
            return;
        }
}

void* Pool::alloc(size_t bytes) {
    bytes = ((bytes ? bytes : 1) + 255) & ~(size_t)255;
    auto it = by_size_.lower_bound(bytes);
    if (it == by_size_.end() && fixed_) throw Error(E_OOM, "fixed scratch region exhausted");
    if (it == by_size_.end()) {
        // new chunk: 8 GiB, or the request rounded up to 1 GiB
        size_t want = std::max(kChunk, (bytes + ((size_t)1 << 30) - 1) & ~(((size_t)1 << 30) - 1));
        void* p = get_chunk(want);
        if (!p) {
            trim(want);
            p = get_chunk(want);
        }
        if (!p && want > bytes) {
            want = bytes;   // as much as the request alone
            p = get_chunk(want);
        }
        if (!p) throw Error(E_OOM, "device allocation failed");
        if (std::getenv("HS_TRACE"))
            std::fprintf(stderr, "[hs] pool: new chunk of %.2f GB (%.2f GB reserved, %.2f GB in use)\n", want / 1e9,
                         (reserved_ + want) / 1e9, in_use_ / 1e9);
        Chunk ch;
        ch.base = (char*)p;
        ch.size = want;
        chunks_.push_back(ch);
        reserved_ += want;
        add_free((int)chunks_.size() - 1, 0, want);
        it = by_size_.lower_bound(bytes);
    }
    const int c = it->second.first;
    const size_t off = it->second.second, size = it->first;
    remove_free(c, off, size);
    if (size > bytes) add_free(c, off + bytes, size - bytes);
    void* p = chunks_[c].base + off;
    live_[p] = std::make_pair(c, bytes);
    in_use_ += bytes;
    return p;
}

void Pool::free(void* p) {
    if (!p) return;
    auto it = live_.find(p);
    if (it == live_.end()) return;
    const int c = it->second.first;
    size_t size = it->second.second;
    size_t off = (size_t)((char*)p - chunks_[c].base);
    live_.erase(it);
    in_use_ -= size;
    auto& fm = chunks_[c].free_;
    // coalesce with the following and the preceding free blocks
    auto nx = fm.find(off + size);
    if (nx != fm.end()) {
        const size_t ns = nx->second;
        remove_free(c, off + size, ns);
        size += ns;
    }
    auto pv = fm.lower_bound(off);
    if (pv != fm.begin()) {
        --pv;
        if (pv->first + pv->second == off) {
            const size_t po = pv->first, ps = pv->second;
            remove_free(c, po, ps);
            off = po;
            size += ps;
        }
    }
    add_free(c, off, size);
}

void Pool::adopt(void* base, size_t bytes) {
    release_all();
    fixed_ = true;
    Chunk ch;
    ch.base = (char*)base;
    ch.size = bytes & ~(size_t)255;
    chunks_.push_back(ch);
    reserved_ = ch.size;
    add_free(0, 0, ch.size);
}

size_t Pool::trim(size_t bytes) {
    // only chunks with no live block can go back to the device
    if (fixed_) return 0;
    size_t released = 0;
    for (int c = (int)chunks_.size() - 1; c >= 0 && released < bytes; c--) {
        Chunk& ch = chunks_[c];
        if (!ch.base) continue;
        auto f = ch.free_.find(0);
        if (f == ch.free_.end() || f->second != ch.size) continue;
        remove_free(c, 0, ch.size);
        put_chunk(ch.base, ch.size);
        released += ch.size;
        reserved_ -= ch.size;
        ch.base = nullptr;
        ch.size = 0;
    }
    return released;
}

void Pool::release_all() {
    if (!fixed_)
        for (auto& ch : chunks_)
            if (ch.base) put_chunk(ch.base, ch.size);
    chunks_.clear();
    by_size_.clear();
    live_.clear();
    in_use_ = reserved_ = 0;
}

Pool::~Pool() { release_all(); }

// --------------------------------------------------------------- context
void Context::sync() {
    HS_REQUIRE(!capturing, E_STATE, "stream synchronisation while a schedule is being captured");
    check_hip(hipStreamSynchronize((hipStream_t)stream), "stream sync");
}

void Context::upload(void* dst, const void* src, size_t bytes) {
    HS_REQUIRE(!capturing, E_STATE, "host-to-device copy while a schedule is being captured");
    check_hip(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, (hipStream_t)stream), "upload");
    sync();
}

void Context::download(void* dst, const void* src, size_t bytes) {
    HS_REQUIRE(!capturing, E_STATE, "device-to-host copy while a schedule is being captured");
    check_hip(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, (hipStream_t)stream), "download");
    sync();
}

void* Context::persistent_alloc(size_t bytes, const char* what) {
    void* p = raw_alloc(bytes, what);
    owned.push_back(p);
    return p;
}

void* Context::raw_alloc(size_t bytes, const char* what) {
    if (bytes == 0) bytes = 8;
    void* p = da.get(bytes);
    if (!p) {
        // the pool's cached blocks may hold the memory
        pool.trim(bytes);
        p = da.get(bytes);
    }
    if (!p) throw Error(E_OOM, std::string("device allocation failed: ") + what);
    raw_sizes[p] = bytes;
    return p;
}

void Context::raw_free(void* p) {
    auto it = raw_sizes.find(p);
    if (it == raw_sizes.end()) return;
    da.put(p, it->second);
    raw_sizes.erase(it);
}

void* Context::dev_table(const void* host, size_t bytes) {
    void* p = persistent_alloc(bytes, "table");
    if (bytes) upload(p, host, bytes);
    return p;
}

RowConsts Context::shoup_consts(const std::vector<u64>& vals, int q_off, bool p_part) const {
    RowConsts rc;
    std::memset(&rc, 0, sizeof(rc));
    HS_REQUIRE(vals.size() <= (size_t)kMaxRows, E_PARAM, "too many rows");
    for (size_t i = 0; i < vals.size(); i++) {
        const u64 qi = p_part ? primes[nq + i] : primes[q_off + i];
        rc.c[i] = vals[i] % qi;
        rc.cs[i] = shoup_h(rc.c[i], qi);
    }
    return rc;
}

Context::Context(const Params& p, int dev, void* st, const DevAllocator* alloc) : prm(p), device(dev) {
    if (alloc) da = *alloc;
    da.stream = st;
    pool.set_source(&da);
    try {
        init();
    } catch (...) {
        release();   // a failed construction returns what it took
        throw;
    }
}

Context::Context(Context& p, void* st) : prm(p.prm), device(p.device) {
    HS_REQUIRE(p.have_keys, E_STATE, "clone: the parent context has no keys yet");
    HS_REQUIRE(!p.parent_ctx, E_ARG, "clone: the parent is itself a clone");
    check_hip(hipSetDevice(device), "hipSetDevice");
    da = p.da;
    da.stream = st;
    pool.set_source(&da);
    stream = st;
    N = p.N;
    logN = p.logN;
    primes = p.primes;
    nq = p.nq;
    np = p.np;
    L = p.L;
    dnum = p.dnum;
    psi = p.psi;
    pinfo = p.pinfo;
    for (int i = 0; i < kMaxRows; i++) P_mod[i] = p.P_mod[i];
    T = p.T;
    T.prof = nullptr;
    tw_cos = p.tw_cos;
    tw_sin = p.tw_sin;
    cdt = p.cdt;
    ncdt = p.ncdt;
    cdt_host = p.cdt_host;
    have_keys = true;
    key_seed = p.key_seed;
    s_coeff = p.s_coeff;
    s_ntt = p.s_ntt;
    pk = p.pk;
    for (auto& kv : p.keys) {
        keys[kv.first] = kv.second;
        borrowed_keys.push_back(kv.first);
    }
    {
        std::lock_guard<std::mutex> g(clone_mutex());
        HS_REQUIRE(!p.destroy_pending, E_STATE, "clone: the parent context has been destroyed");
        parent_ctx = &p;
        p.live_clones++;
    }
    // last, so a clone that fails before holds no profiler; if this fails,
    // the count on the parent is taken back
    try {
        T.prof = prof_create();
    } catch (...) {
        std::lock_guard<std::mutex> g(clone_mutex());
        p.live_clones--;
        parent_ctx = nullptr;
        throw;
    }
}

std::mutex& clone_mutex() {
    static std::mutex m;
    return m;
}

void destroy_context(Context* c) {
    if (!c) return;
    {
        std::lock_guard<std::mutex> g(clone_mutex());
        if (c->live_clones > 0) {
            c->destroy_pending = true;
            return;
        }
    }
    delete c;
}

void Context::init() {
    const Params& p = prm;
    const int dev = device;
    void* st = da.stream;
    HS_REQUIRE(p.logN >= 3 && p.logN <= 17, E_PARAM, "logN out of range");
    HS_REQUIRE(!p.q_bits.empty() && !p.p_bits.empty(), E_PARAM, "need Q and P primes");
    HS_REQUIRE((int)(p.q_bits.size() + p.p_bits.size()) <= kMaxRows, E_PARAM, "too many primes");
    HS_REQUIRE(p.digit >= 1 && p.digit <= 16, E_PARAM, "digit size out of range");
    HS_REQUIRE(p.user_top >= 0 && p.user_top < (int)p.q_bits.size(), E_PARAM, "user_top out of range");
    // the device reductions (Barrett with mu = floor(2^(2b) / q), b = bit
    // length of q) reduce full 64-bit words, which needs 2b >= 64
    for (int b : p.q_bits) HS_REQUIRE(b >= 32 && b <= 61, E_PARAM, "prime sizes must be in [32, 61] bits");
    for (int b : p.p_bits) HS_REQUIRE(b >= 32 && b <= 61, E_PARAM, "prime sizes must be in [32, 61] bits");
    check_hip(hipSetDevice(dev), "hipSetDevice");
    // device address of the allocation-free entry point's scratch array (once
    // per device, with the device current); a failed lookup only disables
    // that entry point
    scratch_init(dev);
    stream = st;
    logN = p.logN;
    N = 1 << logN;
    nq = (int)p.q_bits.size();
    np = (int)p.p_bits.size();
    L = nq - 1;
    dnum = (nq + p.digit - 1) / p.digit;
    HS_REQUIRE(dnum <= 16, E_PARAM, "too many digits");
    std::vector<int> bits = p.q_bits;
    bits.insert(bits.end(), p.p_bits.begin(), p.p_bits.end());
    primes = find_primes(logN, bits);
    // every key-switching digit must be far below P: the switching noise is
    // about (digit / P) * (primes per digit) * sigma * sqrt(N) per coefficient
    // on top of the ModDown rounding, and it lands on the raw message (in
    // bootstrapping, before CoeffToSlot has scaled anything up); a 2^20
    // margin keeps it below the rounding term
    double logP = 0;
    for (int k = 0; k < np; k++) logP += std::log2((double)primes[nq + k]);
    for (int j = 0; j < dnum; j++) {
        double lg = 0;
        for (int i = j * p.digit; i < std::min(nq, (j + 1) * p.digit); i++) lg += std::log2((double)primes[i]);
        HS_REQUIRE(lg + 20.0 <= logP, E_PARAM, "a key-switching digit is not 2^20 below the special modulus P");
    }
    const int nt = nq + np;
    pinfo.resize(nt);
    psi.resize(nt);
    std::vector<u64> tw((size_t)nt * N), tws((size_t)nt * N), itw((size_t)nt * N), itws((size_t)nt * N),
        ninv(2 * (size_t)nt);
    for (int t = 0; t < nt; t++) {
        const u64 qt = primes[t];
        int b = 0;
        while ((qt >> b) != 0) b++;
        pinfo[t].q = qt;
        pinfo[t].bits = b;
        pinfo[t].mu = (u64)(((u128)1 << (2 * b)) / qt);
        pinfo[t].nq = 0 - qt;
        psi[t] = smallest_psi(qt, N);
        const u64 pinv = invmod_h(psi[t], qt);
        // powers by bit-reversed exponent
        std::vector<u64> pw(N), ipw(N);
        pw[0] = ipw[0] = 1;
        for (int k = 1; k < N; k++) {
            pw[k] = mulmod_h(pw[k - 1], psi[t], qt);
            ipw[k] = mulmod_h(ipw[k - 1], pinv, qt);
        }
        for (int k = 0; k < N; k++) {
            const u64 e = brv((u64)k, logN);
            tw[(size_t)t * N + k] = pw[e];
            tws[(size_t)t * N + k] = shoup_h(pw[e], qt);
            itw[(size_t)t * N + k] = ipw[e];
            itws[(size_t)t * N + k] = shoup_h(ipw[e], qt);
        }
        ninv[2 * t] = invmod_h((u64)N % qt, qt);
        ninv[2 * t + 1] = shoup_h(ninv[2 * t], qt);
    }
    for (int i = 0; i < nq; i++) {
        u64 pm = 1;
        for (int k = 0; k < np; k++) pm = mulmod_h(pm, primes[nq + k] % primes[i], primes[i]);
        P_mod[i] = pm;
    }
    T.prime = (const PrimeInfo*)dev_table(pinfo.data(), sizeof(PrimeInfo) * nt);
    T.tw = (const u64*)dev_table(tw.data(), tw.size() * 8);
    T.tws = (const u64*)dev_table(tws.data(), tws.size() * 8);
    T.itw = (const u64*)dev_table(itw.data(), itw.size() * 8);
    T.itws = (const u64*)dev_table(itws.data(), itws.size() * 8);
    T.ninv = (const u64*)dev_table(ninv.data(), ninv.size() * 8);
    {
        std::vector<u64> a(2 * (size_t)nt * N), b(2 * (size_t)nt * N);
        for (size_t k = 0; k < (size_t)nt * N; k++) {
            a[2 * k] = tw[k];
            a[2 * k + 1] = tws[k];
            b[2 * k] = itw[k];
            b[2 * k + 1] = itws[k];
        }
        T.tw2 = (const u64*)dev_table(a.data(), a.size() * 8);
        std::vector<u64> r64(nt);
        for (int t = 0; t < nt; t++) r64[t] = (u64)(((u128)1 << 64) % primes[t]);
        T.r64 = (const u64*)dev_table(r64.data(), r64.size() * 8);
        T.itw2 = (const u64*)dev_table(b.data(), b.size() * 8);
    }
    T.logN = logN;
    T.N = N;
    T.prof = prof_create();

    // encoding twiddles: correctly rounded (cos, sin)(pi e / N), e in [0, 2N),
    // from binary128 values on the quarter circle and exact symmetries
    const int quarter = N / 2;
    std::vector<double> c(quarter + 1);
    for (int e = 0; e <= quarter; e++) {
        if (e == quarter) {
            c[e] = 0.0;  // cos(pi/2)
        } else {
            __float128 a = M_PIq * (__float128)e / (__float128)N;
            c[e] = (double)cosq(a);
        }
    }
    tw_cos.resize(2 * N);
    tw_sin.resize(2 * N);
    for (int e = 0; e < 2 * N; e++) {
        double cr, sr;
        if (e <= quarter) {
            cr = c[e];
            sr = c[quarter - e];
        } else if (e <= N) {
            int f = e - quarter;
            cr = -c[quarter - f];
            sr = c[f];
        } else if (e <= N + quarter) {
            int f = e - N;
            cr = -c[f];
            sr = -c[quarter - f];
        } else {
            int f = e - N - quarter;
            cr = c[quarter - f];
            sr = -c[f];
        }
        tw_cos[e] = cr;
        tw_sin[e] = sr;
    }

    // discrete Gaussian table: floor(2^64 Pr(|e| <= k)), k < 40, last = 2^64-1
    {
        const int kmax = 40;
        const __float128 s2 = 2 * (__float128)p.sigma * (__float128)p.sigma;
        std::vector<__float128> rho(200);
        for (int k = 0; k < 200; k++) rho[k] = expq(-((__float128)k * k) / s2);
        __float128 Z = rho[0];
        for (int k = 1; k < 200; k++) Z += 2 * rho[k];
        cdt_host.resize(kmax);
        __float128 acc = rho[0];
        const __float128 two64 = ldexpq(1.0Q, 64);
        for (int k = 0; k < kmax; k++) {
            if (k > 0) acc += 2 * rho[k];
            __float128 v = floorq(acc / Z * two64);
            cdt_host[k] = v >= two64 ? ~0ull : (u64)v;
        }
        cdt_host[kmax - 1] = ~0ull;
        ncdt = kmax;
        cdt = (u64*)dev_table(cdt_host.data(), cdt_host.size() * 8);
    }
}

Context::~Context() { release(); }

void Context::release() {
    // pending work may still read the blocks
    if (stream || T.prof) (void)hipStreamSynchronize((hipStream_t)stream);
    boot_release(this);
    prof_destroy(T.prof);
    T.prof = nullptr;
    for (auto& kv : keys)
        if (std::find(borrowed_keys.begin(), borrowed_keys.end(), kv.first) == borrowed_keys.end())
            pool.free(kv.second);
    keys.clear();
    borrowed_keys.clear();
    if (!parent_ctx) {
        if (s_ntt) pool.free(s_ntt);
        if (pk) pool.free(pk);
    }
    s_ntt = pk = nullptr;
    if (parent_ctx) {
        Context* orphan = nullptr;
        {
            std::lock_guard<std::mutex> g(clone_mutex());
            if (--parent_ctx->live_clones == 0 && parent_ctx->destroy_pending) orphan = parent_ctx;
        }
        parent_ctx = nullptr;
        delete orphan;   // its owner destroyed it while this clone lived
    }
    pool.release_all();
    for (void* p : owned) raw_free(p);
    owned.clear();
    for (auto& kv : perms) raw_free(kv.second);
    perms.clear();
    for (auto& kv : modup)
        for (void* p : kv.second.bufs) raw_free(p);
    modup.clear();
    for (auto& kv : moddown)
        for (void* p : kv.second.bufs) raw_free(p);
    moddown.clear();
    mask_pts.clear();
    monomials.clear();
    for (auto& kv : raw_sizes) da.put(kv.first, kv.second);   // anything else raw_alloc gave out
    raw_sizes.clear();
}

CtHandle::~CtHandle() {
    if (ctx && ct.d) ctx->free_words(ct.d);
}

// ------------------------------------------------- base-conversion tables
static ConvDev make_conv(Context& c, const std::vector<int>& src, const std::vector<int>& src_row,
                         const std::vector<int>& dst, const std::vector<int>& dst_row, bool centered,
                         const std::vector<int>& own_row = {}, const std::vector<u64>& post = {}) {
    const int k = (int)src.size(), m = (int)dst.size();
    // the conversion kernel holds k sources in registers and m targets in LDS
    HS_REQUIRE(k >= 1 && k <= 16 && m <= kMaxRows, E_PARAM, "base conversion shape out of range");
    std::vector<u64> inv_hat(k), inv_hat_s(k), hat((size_t)k * m), hat_s((size_t)k * m);
    for (int i = 0; i < k; i++) {
        const u64 di = c.primes[src[i]];
        u64 h = 1;
        for (int j = 0; j < k; j++)
            if (j != i) h = mulmod_h(h, c.primes[src[j]] % di, di);
        inv_hat[i] = invmod_h(h, di);
        inv_hat_s[i] = shoup_h(inv_hat[i], di);
        for (int t = 0; t < m; t++) {
            const u64 qt = c.primes[dst[t]];
            u64 g = 1;
            for (int j = 0; j < k; j++)
                if (j != i) g = mulmod_h(g, c.primes[src[j]] % qt, qt);
            if (!post.empty()) g = mulmod_h(g, post[t], qt);   // output times post[t]
            hat[(size_t)i * m + t] = g;
            hat_s[(size_t)i * m + t] = shoup_h(g, qt);
        }
    }
    ConvDev cd;
    auto put = [&](const void* h, size_t bytes) {
        void* p = c.raw_alloc(bytes, "conversion table");
        if (bytes) c.upload(p, h, bytes);
        cd.bufs.push_back(p);
        return p;
    };
    cd.t.inv_hat = (const u64*)put(inv_hat.data(), k * 8);
    cd.t.inv_hat_s = (const u64*)put(inv_hat_s.data(), k * 8);
    cd.t.hat = (const u64*)put(hat.data(), hat.size() * 8);
    cd.t.hat_s = (const u64*)put(hat_s.data(), hat_s.size() * 8);
    cd.t.src_prime = (const int*)put(src.data(), k * 4);
    cd.t.dst_prime = (const int*)put(dst.data(), m * 4);
    cd.t.src_row = (const int*)put(src_row.data(), k * 4);
    cd.t.dst_row = (const int*)put(dst_row.data(), m * 4);
    cd.t.own_row = nullptr;
    if (!own_row.empty()) {
        HS_REQUIRE((int)own_row.size() == k, E_PARAM, "one own row per source");
        cd.t.own_row = (const int*)put(own_row.data(), k * 4);
    }
    std::vector<u64> dmod(m);
    for (int t = 0; t < m; t++) {
        const u64 qt = c.primes[dst[t]];
        u64 g = 1;
        for (int j = 0; j < k; j++) g = mulmod_h(g, c.primes[src[j]] % qt, qt);
        if (!post.empty()) g = mulmod_h(g, post[t], qt);
        dmod[t] = g;
    }
    cd.t.dmod = (const u64*)put(dmod.data(), m * 8);
    std::vector<u64> r64(m), r64s(m), ones(m);
    for (int t = 0; t < m; t++) {
        const u64 qt = c.primes[dst[t]];
        r64[t] = (u64)(((u128)1 << 64) % qt);
        r64s[t] = shoup_h(r64[t], qt);
        ones[t] = shoup_h(1, qt);
    }
    cd.t.r64 = (const u64*)put(r64.data(), m * 8);
    cd.t.r64s = (const u64*)put(r64s.data(), m * 8);
    cd.t.ones = (const u64*)put(ones.data(), m * 8);
    cd.t.k = k;
    cd.t.m = m;
    cd.t.centered = centered ? 1 : 0;
    // byte-plane tables for the matrix-core kernel: the balanced base-256
    // digits of v < 2^62 are the bytes of (v + c) xor c, c = 0x80..80, and the
    // plane sums stay exact in int32 when targets are in [2^39, 2^62)
    cd.t.bfrag = nullptr;
    cd.t.c48 = cd.t.c48s = nullptr;
    cd.t.nks = (k + 3) / 4;
    cd.t.ntb = (m + 15) / 16;
    bool planes_ok = k <= 16;
    for (int i : src) planes_ok = planes_ok && c.primes[i] < (1ull << 62);
    for (int t : dst) planes_ok = planes_ok && c.primes[t] >= (1ull << 39) && c.primes[t] < (1ull << 62);
    if (planes_ok) {
        const u64 bias = 0x8080808080808080ull;
        const int nks = cd.t.nks, ntb = cd.t.ntb;
        std::vector<u64> bf((size_t)ntb * nks * 8 * 64, 0);
        for (int tb = 0; tb < ntb; tb++)
            for (int ks = 0; ks < nks; ks++)
                for (int lane = 0; lane < 64; lane++) {
                    const int t = tb * 16 + (lane & 15), i = 4 * ks + (lane >> 4);
                    if (t >= m || i >= k) continue;
                    const u64 qt = c.primes[dst[t]];
                    for (int a = 0; a < 8; a++) {
                        const u64 H = mulmod_h(powmod_h(2, 8 * a, qt), hat[(size_t)i * m + t], qt);
                        const u64 Hd = (H + bias) ^ bias;
                        for (int b = 0; b < 8; b++)
                            bf[((size_t)(tb * nks + ks) * 8 + b) * 64 + lane] |= ((Hd >> (8 * b)) & 0xff) << (8 * a);
                    }
                }
        std::vector<u64> c48(m), c48s(m);
        for (int t = 0; t < m; t++) {
            const u64 qt = c.primes[dst[t]];
            c48[t] = powmod_h(2, 48, qt);
            c48s[t] = shoup_h(c48[t], qt);
        }
        cd.t.bfrag = (const u64*)put(bf.data(), bf.size() * 8);
        cd.t.c48 = (const u64*)put(c48.data(), m * 8);
        cd.t.c48s = (const u64*)put(c48s.data(), m * 8);
    }
    return cd;
}

// ModUp of digit j at level l: sources are the digit's primes (rows = prime
// index in a level-l polynomial), targets are every other prime of
// q_0..q_l and all of P, written to rows of the extended layout
// (Q rows 0..l, then P rows l+1..l+alpha).
const ConvDev& Context::modup_tables(int level, int j) {
    auto key = std::make_pair(level, j);
    auto it = modup.find(key);
    if (it != modup.end()) return it->second;
    std::vector<int> src, srow, dst, drow;
    const int lo = j * prm.digit, hi = std::min((j + 1) * prm.digit, level + 1);
    for (int i = lo; i < hi; i++) {
        src.push_back(i);
        srow.push_back(i);
    }
    for (int i = 0; i <= level; i++)
        if (i < lo || i >= hi) {
            dst.push_back(i);
            drow.push_back(i);
        }
    for (int k = 0; k < np; k++) {
        dst.push_back(nq + k);
        drow.push_back(level + 1 + k);
    }
    HS_REQUIRE((int)src.size() <= 16, E_PARAM, "digit too large");
    // the digit's own rows go to the same rows of the extended layout unchanged
    return modup.emplace(key, make_conv(*this, src, srow, dst, drow, false, srow)).first->second;
}

// ModDown at level l: sources are P (rows l+1.. of the extended layout),
// targets q_0..q_l (rows 0..l of a level-l buffer).  Centred conversion, so
// the division by P rounds with a zero-mean error.
const ConvDev& Context::moddown_tables(int level) {
    auto it = moddown.find(level);
    if (it != moddown.end()) return it->second;
    std::vector<int> src, srow, dst, drow;
    for (int k = 0; k < np; k++) {
        src.push_back(nq + k);
        srow.push_back(level + 1 + k);
    }
    for (int i = 0; i <= level; i++) {
        dst.push_back(i);
        drow.push_back(i);
    }
    HS_REQUIRE((int)src.size() <= 16, E_PARAM, "too many special primes");
    // outputs come out times P^-1 (the key's Q rows carry the same factor)
    std::vector<u64> pinv(level + 1);
    for (int i = 0; i <= level; i++) pinv[i] = invmod_h(P_mod[i], primes[i]);
    return moddown.emplace(level, make_conv(*this, src, srow, dst, drow, true, {}, pinv)).first->second;
}

// X -> X^g in the bit-reversed NTT domain: out[i] = in[perm[i]] with
// 2 brv(perm[i]) + 1 = (2 brv(i) + 1) g mod 2N.
const int* Context::perm(int g) {
    auto it = perms.find(g);
    if (it != perms.end()) return it->second;
    std::vector<int> p(N);
    const u64 M = 2 * (u64)N;
    for (int i = 0; i < N; i++) {
        const u64 e = ((2 * brv((u64)i, logN) + 1) * (u64)g) % M;
        p[i] = (int)brv((e - 1) / 2, logN);
    }
    int* d = (int*)raw_alloc(sizeof(int) * N, "permutation");
    upload(d, p.data(), sizeof(int) * N);
    perms[g] = d;
    return d;
}

// ---------------------------------------------------------- ciphertexts
Ct ct_alloc(Context& c, int m, int ncomp, int level) {
    HS_REQUIRE(level >= 0 && level <= c.L, E_LEVEL, "level out of range");
    Ct a;
    a.m = m;
    a.ncomp = ncomp;
    a.level = level;
    a.d = c.alloc_words((size_t)m * a.ct_words(c.N));
    return a;
}

void ct_free(Context& c, Ct& a) {
    if (a.d) c.free_words(a.d);
    a.d = nullptr;
}

Ct ct_copy(Context& c, const Ct& a) {
    Ct o = ct_alloc(c, a.m, a.ncomp, a.level);
    o.scale = a.scale;
    k_copy_rows(c.T, c.ct_rows(o), c.ct_rows(a), c.stream);
    return o;
}

Ct ct_drop(Context& c, const Ct& a, int level) {
    HS_REQUIRE(level <= a.level && level >= 0, E_LEVEL, "cannot drop to a higher level");
    Ct o = ct_alloc(c, a.m, a.ncomp, level);
    o.scale = a.scale;
    Rows in = c.ct_rows(a);
    in.rpg = level + 1;
    in.nq = level + 1;
    k_copy_rows(c.T, c.ct_rows(o), in, c.stream);
    return o;
}

Ct ct_slice(Context& c, const Ct& a, int first, int count) {
    Ct o = ct_alloc(c, count, a.ncomp, a.level);
    o.scale = a.scale;
    Rows in = c.ct_rows(o);
    in.base = a.d + (size_t)first * a.ct_words(c.N);
    k_copy_rows(c.T, c.ct_rows(o), in, c.stream);
    return o;
}

Ct ct_gather(Context& c, const std::vector<const Ct*>& parts) {
    HS_REQUIRE(!parts.empty(), E_ARG, "empty gather");
    int m = 0;
    for (auto* p : parts) {
        HS_REQUIRE(p->level == parts[0]->level && p->ncomp == parts[0]->ncomp, E_LEVEL,
                   "gathered ciphertexts must share level and size");
        m += p->m;
    }
    Ct o = ct_alloc(c, m, parts[0]->ncomp, parts[0]->level);
    o.scale = parts[0]->scale;
    size_t off = 0;
    for (auto* p : parts) {
        Rows out = c.ct_rows(*p);
        out.base = o.d + off;
        k_copy_rows(c.T, out, c.ct_rows(*p), c.stream);
        off += (size_t)p->m * p->ct_words(c.N);
    }
    return o;
}

// ------------------------------------------------------------ sampling
// Domain tags of the Philox draws (bits 56..63 = purpose).
static const u64 D_SECRET = 1ull << 56, D_PK_A = 2ull << 56, D_PK_E = 3ull << 56, D_KEY_A = 4ull << 56,
                 D_KEY_E = 5ull << 56, D_ENC_V = 6ull << 56, D_ENC_E0 = 7ull << 56, D_ENC_E1 = 8ull << 56;

static void philox_host(u64 seed, u64 domain, u64 index, u32 out[4]) {
    u32 c0 = (u32)index, c1 = (u32)(index >> 32), c2 = (u32)domain, c3 = (u32)(domain >> 32);
    u32 k0 = (u32)seed, k1 = (u32)(seed >> 32);
    for (int r = 0; r < 10; r++) {
        u64 p0 = (u64)0xD2511F53u * c0;
        u64 p1 = (u64)0xCD9E8D57u * c2;
        u32 n0 = (u32)(p1 >> 32) ^ c1 ^ k0;
        u32 n1 = (u32)p1;
        u32 n2 = (u32)(p0 >> 32) ^ c3 ^ k1;
        u32 n3 = (u32)p0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

static std::vector<int64_t> sample_secret(const Context& c, u64 seed) {
    std::vector<int64_t> s(c.N, 0);
    if (c.prm.hamming == 0) {
        for (int i = 0; i < c.N; i++) {
            u32 w[4];
            philox_host(seed, D_SECRET, (u64)i, w);
            u32 r = w[0] % 3u;
            s[i] = r == 0 ? 0 : (r == 1 ? 1 : -1);
        }
    } else {
        HS_REQUIRE(c.prm.hamming <= c.N, E_PARAM, "Hamming weight exceeds N");
        std::vector<u64> pos(c.N);
        for (int i = 0; i < c.N; i++) pos[i] = i;
        for (int t = 0; t < c.prm.hamming; t++) {
            u32 w[4];
            philox_host(seed, D_SECRET, (u64)t, w);
            u64 r = ((u64)w[1] << 32) | w[0];
            u64 j = t + r % (u64)(c.N - t);
            std::swap(pos[t], pos[j]);
            s[pos[t]] = (w[2] & 1u) ? -1 : 1;
        }
    }
    return s;
}

// NTT-domain rows (rows of q_off.. / P) of a small polynomial sampled on device
static void small_poly_rows(Context& c, const Rows& out, u64 seed, u64 domain, int kind) {
    int64_t* tmp = (int64_t*)c.pool.alloc(sizeof(int64_t) * c.N);
    k_sample_small(tmp, c.N, seed, domain, kind, c.cdt, c.ncdt, c.stream);
    k_small_to_rows(c.T, out, tmp, c.stream);
    k_ntt(c.T, out, false, c.stream);
    c.sync();
    c.pool.free(tmp);
}

static u64* make_switch_key(Context& c, int key_id, const u64* s_target) {
    const int nt = c.nq + c.np;
    const size_t rows_words = (size_t)nt * c.N;
    u64* key = c.alloc_words((size_t)c.dnum * 2 * rows_words);
    u64* tmp = c.alloc_words(rows_words);
    for (int j = 0; j < c.dnum; j++) {
        u64* b = key + (size_t)(2 * j) * rows_words;
        u64* a = key + (size_t)(2 * j + 1) * rows_words;
        Rows ra{a, 1, nt, rows_words, c.nq, 0, c.nq};
        Rows rb{b, 1, nt, rows_words, c.nq, 0, c.nq};
        Rows rs{c.s_ntt, 1, nt, rows_words, c.nq, 0, c.nq};
        Rows rt{tmp, 1, nt, rows_words, c.nq, 0, c.nq};
        k_sample_uniform(c.T, ra, c.key_seed, D_KEY_A | ((u64)key_id << 24) | ((u64)j << 16), c.stream);
        small_poly_rows(c, rb, c.key_seed, D_KEY_E | ((u64)key_id << 24) | ((u64)j << 16), 2);
        k_mul(c.T, rt, ra, rs, c.stream);
        k_sub(c.T, rb, rb, rt, c.stream);
        const int lo = j * c.prm.digit, hi = std::min((j + 1) * c.prm.digit, c.nq);
        std::vector<u64> pm;
        for (int i = lo; i < hi; i++) pm.push_back(c.P_mod[i]);
        RowConsts rc = c.shoup_consts(pm, lo);
        Rows dst{b + (size_t)lo * c.N, 1, hi - lo, rows_words, hi - lo, lo, c.nq};
        Rows st{const_cast<u64*>(s_target) + (size_t)lo * c.N, 1, hi - lo, rows_words, hi - lo, lo, c.nq};
        Rows t2{tmp, 1, hi - lo, rows_words, hi - lo, lo, c.nq};
        k_mul_row_const(c.T, t2, st, rc, c.stream);
        k_add(c.T, dst, dst, t2, c.stream);
    }
    // stored with the Q rows times P^-1 mod q_i: the inner product then lands
    // divided by P on Q, and ModDown only subtracts (the P rows, which feed
    // the ModDown conversion, are kept as they are); hs_key_export undoes it
    std::vector<u64> pinv(c.nq);
    for (int i = 0; i < c.nq; i++) pinv[i] = invmod_h(c.P_mod[i], c.primes[i]);
    Rows rq{key, 2 * c.dnum, c.nq, rows_words, c.nq, 0, c.nq};
    k_mul_row_const(c.T, rq, rq, c.shoup_consts(pinv, 0), c.stream);
    c.sync();
    c.free_words(tmp);
    return key;
}

void keygen(Context& c, u64 seed) {
    HS_REQUIRE(!c.parent_ctx, E_STATE, "keygen: a clone uses its parent's keys");
    {
        std::lock_guard<std::mutex> g(clone_mutex());
        HS_REQUIRE(c.live_clones == 0, E_STATE, "keygen: contexts cloned from this one still use its keys");
    }
    ContextArena arena(c);
    const int nt = c.nq + c.np;
    const size_t rows_words = (size_t)nt * c.N;
    for (auto& kv : c.keys) c.free_words(kv.second);
    c.keys.clear();
    if (c.s_ntt) c.free_words(c.s_ntt);
    if (c.pk) c.free_words(c.pk);
    c.key_seed = seed;
    c.s_coeff = sample_secret(c, seed);
    c.s_ntt = c.alloc_words(rows_words);
    {
        int64_t* tmp = (int64_t*)c.pool.alloc(sizeof(int64_t) * c.N);
        c.upload(tmp, c.s_coeff.data(), sizeof(int64_t) * c.N);
        Rows rs{c.s_ntt, 1, nt, rows_words, c.nq, 0, c.nq};
        k_small_to_rows(c.T, rs, tmp, c.stream);
        k_ntt(c.T, rs, false, c.stream);
        c.sync();
        c.pool.free(tmp);
    }
    // public key (b, a) = (-a s + e, a) over Q
    c.pk = c.alloc_words(2 * (size_t)c.nq * c.N);
    {
        const size_t qw = (size_t)c.nq * c.N;
        Rows r0 = c.rows(c.pk, 1, c.nq, qw), r1 = c.rows(c.pk + qw, 1, c.nq, qw);
        Rows rs = c.rows(c.s_ntt, 1, c.nq, qw);
        k_sample_uniform(c.T, r1, seed, D_PK_A, c.stream);
        small_poly_rows(c, r0, seed, D_PK_E, 2);
        u64* tmp = c.alloc_words(qw);
        Rows rt = c.rows(tmp, 1, c.nq, qw);
        k_mul(c.T, rt, r1, rs, c.stream);
        k_sub(c.T, r0, r0, rt, c.stream);
        c.sync();
        c.free_words(tmp);
    }
    // relinearisation key: target s^2
    u64* s2 = c.alloc_words(rows_words);
    {
        Rows rs{c.s_ntt, 1, nt, rows_words, c.nq, 0, c.nq};
        Rows r2{s2, 1, nt, rows_words, c.nq, 0, c.nq};
        k_mul(c.T, r2, rs, rs, c.stream);
    }
    c.keys[0] = make_switch_key(c, 0, s2);
    c.free_words(s2);
    c.have_keys = true;
}

void add_galois_key(Context& c, int g) {
    HS_REQUIRE(c.have_keys, E_STATE, "keygen first");
    g = ((g % (2 * c.N)) + 2 * c.N) % (2 * c.N);
    HS_REQUIRE(g % 2 == 1, E_ARG, "Galois element must be odd");
    if (c.keys.count(g)) return;
    ContextArena arena(c);
    const int nt = c.nq + c.np;
    const size_t rows_words = (size_t)nt * c.N;
    u64* sg = c.alloc_words(rows_words);
    Rows rs{c.s_ntt, 1, nt, rows_words, c.nq, 0, c.nq};
    Rows rg{sg, 1, nt, rows_words, c.nq, 0, c.nq};
    k_permute(c.T, rg, rs, c.perm(g), c.stream);
    c.keys[g] = make_switch_key(c, g, sg);
    c.free_words(sg);
}

bool has_key(const Context& c, int id) { return c.keys.count(id) != 0; }

// --------------------------------------------------------------- encoding
static int stage_exp(int N, int length, int j, std::vector<int>& cache) {
    (void)j;
    (void)N;
    (void)length;
    return cache[j];
}

static void stage_exponents(int N, int length, std::vector<int>& e) {
    const int h = length / 2;
    const long long lq = 4LL * length;
    e.resize(h);
    long long p = 1;
    for (int j = 0; j < h; j++) {
        e[j] = (int)(p * (2LL * N / lq));
        p = p * 5 % lq;
    }
}

static std::vector<int> brv_perm(int n) {
    int bits = 0;
    while ((1 << bits) < n) bits++;
    std::vector<int> r(n);
    for (int i = 0; i < n; i++) r[i] = (int)brv((u64)i, bits);
    return r;
}

// w = U^-1 z (encode direction).  Butterfly (a, b) -> (a + b, (a - b) conj(W))
// with every product and sum a separately rounded double operation; then bit
// reversal and multiplication by 2^-log2(N/2).
void special_fft_inverse(const Context& c, std::vector<double>& re, std::vector<double>& im) {
    const int n = c.N / 2;
    std::vector<int> e;
    for (int length = n; length >= 2; length /= 2) {
        const int h = length / 2;
        stage_exponents(c.N, length, e);
        for (int base = 0; base < n; base += length) {
            for (int j = 0; j < h; j++) {
                const double cw = c.tw_cos[e[j]], sw = c.tw_sin[e[j]];
                const double ar = re[base + j], ai = im[base + j];
                const double br = re[base + j + h], bi = im[base + j + h];
                const double ur = ar + br, ui = ai + bi;
                const double dr = ar - br, di = ai - bi;
                const double p1 = dr * cw, p2 = di * sw, p3 = di * cw, p4 = dr * sw;
                re[base + j] = ur;
                im[base + j] = ui;
                re[base + j + h] = p1 + p2;
                im[base + j + h] = p3 - p4;
            }
        }
    }
    std::vector<int> perm = brv_perm(n);
    std::vector<double> r2(n), i2(n);
    const double scale = 1.0 / n;
    for (int i = 0; i < n; i++) {
        r2[i] = re[perm[i]] * scale;
        i2[i] = im[perm[i]] * scale;
    }
    re.swap(r2);
    im.swap(i2);
}

// z = U w (decode direction).
void special_fft(const Context& c, std::vector<double>& re, std::vector<double>& im) {
    const int n = c.N / 2;
    std::vector<int> perm = brv_perm(n);
    std::vector<double> r2(n), i2(n);
    for (int i = 0; i < n; i++) {
        r2[i] = re[perm[i]];
        i2[i] = im[perm[i]];
    }
    re.swap(r2);
    im.swap(i2);
    std::vector<int> e;
    for (int length = 2; length <= n; length *= 2) {
        const int h = length / 2;
        stage_exponents(c.N, length, e);
        for (int base = 0; base < n; base += length) {
            for (int j = 0; j < h; j++) {
                const double cw = c.tw_cos[e[j]], sw = c.tw_sin[e[j]];
                const double br = re[base + j + h], bi = im[base + j + h];
                const double p1 = br * cw, p2 = bi * sw, p3 = br * sw, p4 = bi * cw;
                const double tr = p1 - p2, ti = p3 + p4;
                const double ar = re[base + j], ai = im[base + j];
                re[base + j] = ar + tr;
                im[base + j] = ai + ti;
                re[base + j + h] = ar - tr;
                im[base + j + h] = ai - ti;
            }
        }
    }
}

void encode_to(Context& c, u64* out, const double* re, const double* im, int level, double scale) {
    const int n = c.N / 2;
    std::vector<double> r(re, re + n), i(n, 0.0);
    if (im) i.assign(im, im + n);
    special_fft_inverse(c, r, i);
    std::vector<double> w(c.N);
    for (int k = 0; k < n; k++) {
        w[k] = r[k];
        w[k + n] = i[k];
    }
    double* dw = (double*)c.pool.alloc(sizeof(double) * c.N);
    c.upload(dw, w.data(), sizeof(double) * c.N);
    Rows o = c.rows(out, 1, level + 1, (size_t)(level + 1) * c.N);
    k_encode_real(c.T, o, dw, 0, scale, c.stream);
    k_ntt(c.T, o, false, c.stream);
    c.sync();
    c.pool.free(dw);
}

Ct encrypt(Context& c, const u64* pt, int level, double scale, u64 seed) {
    HS_REQUIRE(c.have_keys, E_STATE, "keygen first");
    HS_REQUIRE(level >= 0 && level <= c.L, E_LEVEL, "level out of range");
    Ct ct = ct_alloc(c, 1, 2, level);
    ct.scale = scale;
    const size_t lw = (size_t)(level + 1) * c.N;
    const size_t qw = (size_t)c.nq * c.N;
    u64* v = c.alloc_words(lw);
    u64* e = c.alloc_words(lw);
    Rows rv = c.rows(v, 1, level + 1, lw), re = c.rows(e, 1, level + 1, lw);
    Rows c0 = c.comp_rows(ct, 0), c1 = c.comp_rows(ct, 1);
    Rows pk0 = c.rows(c.pk, 1, level + 1, qw), pk1 = c.rows(c.pk + qw, 1, level + 1, qw);
    Rows rp = c.rows(const_cast<u64*>(pt), 1, level + 1, lw);
    small_poly_rows(c, rv, seed, D_ENC_V, 0);
    small_poly_rows(c, re, seed, D_ENC_E0, 2);
    k_mul(c.T, c0, rv, pk0, c.stream);
    k_add(c.T, c0, c0, re, c.stream);
    k_add(c.T, c0, c0, rp, c.stream);
    small_poly_rows(c, re, seed, D_ENC_E1, 2);
    k_mul(c.T, c1, rv, pk1, c.stream);
    k_add(c.T, c1, c1, re, c.stream);
    c.sync();
    c.free_words(v);
    c.free_words(e);
    return ct;
}

// Coefficients (as doubles, before division by the scale) of the decryption
// of ciphertext `index` of the batch, from the CRT of q_0 and (if present) q_1.
std::vector<double> decrypt_coeffs_double(Context& c, const Ct& a, int index) {
    HS_REQUIRE(c.have_keys, E_STATE, "keygen first");
    HS_REQUIRE(index >= 0 && index < a.m, E_ARG, "index out of range");
    const int nr = std::min(a.level, 1) + 1;
    const size_t lw = (size_t)nr * c.N;
    const size_t nt_w = (size_t)(c.nq + c.np) * c.N;
    u64* acc = c.alloc_words(lw);
    u64* tmp = c.alloc_words(lw);
    u64* sp = c.alloc_words(lw);
    Rows ra = c.rows(acc, 1, nr, lw), rt = c.rows(tmp, 1, nr, lw), rsp = c.rows(sp, 1, nr, lw);
    Rows rs = c.rows(c.s_ntt, 1, nr, nt_w);
    const u64* base = a.d + (size_t)index * a.ct_words(c.N);
    k_copy_rows(c.T, ra, c.rows(const_cast<u64*>(base), 1, nr, lw), c.stream);
    k_copy_rows(c.T, rsp, rs, c.stream);
    for (int k = 1; k < a.ncomp; k++) {
        Rows ck = c.rows(const_cast<u64*>(base) + (size_t)k * a.comp_words(c.N), 1, nr, lw);
        k_mul(c.T, rt, ck, rsp, c.stream);
        k_add(c.T, ra, ra, rt, c.stream);
        if (k + 1 < a.ncomp) k_mul(c.T, rsp, rsp, rs, c.stream);
    }
    k_ntt(c.T, ra, true, c.stream);
    std::vector<u64> h(lw);
    c.download(h.data(), acc, lw * 8);
    c.free_words(acc);
    c.free_words(tmp);
    c.free_words(sp);
    std::vector<double> out(c.N);
    const u64 q0 = c.primes[0];
    if (nr == 1) {
        for (int i = 0; i < c.N; i++) {
            u64 x = h[i];
            out[i] = x > (q0 - 1) / 2 ? -(double)(q0 - x) : (double)x;
        }
    } else {
        const u64 q1 = c.primes[1];
        const u64 q0inv = invmod_h(q0 % q1, q1);
        const u128 Q = (u128)q0 * q1;
        for (int i = 0; i < c.N; i++) {
            const u64 x0 = h[i], x1 = h[c.N + i];
            const u64 d = mulmod_h((x1 + q1 - x0 % q1) % q1, q0inv, q1);
            const u128 x = (u128)x0 + (u128)q0 * d;
            if (x > Q / 2) out[i] = -(double)(Q - x);
            else out[i] = (double)x;
        }
    }
    return out;
}

void decrypt_decode(Context& c, const Ct& a, int index, double* re, double* im) {
    std::vector<double> coef = decrypt_coeffs_double(c, a, index);
    const int n = c.N / 2;
    std::vector<double> r(n), i(n);
    for (int k = 0; k < n; k++) {
        r[k] = coef[k] / a.scale;
        i[k] = coef[k + n] / a.scale;
    }
    special_fft(c, r, i);
    for (int k = 0; k < n; k++) {
        re[k] = r[k];
        if (im) im[k] = i[k];
    }
}

}  // namespace hs
