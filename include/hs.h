/*
 * hs.h -- C ABI of the MI355X homomorphic Softmax library.
 *
 * The library evaluates Softmax on RNS-CKKS ciphertexts by the
 * normalize-and-square method of Cho, Hanrot, Kim, Park and Stehle, "Fast and
 * Accurate Homomorphic Softmax Evaluation" (CCS'24): Algorithm "SM"
 * (Section 3.2), the auxiliary thread (Algorithm "alg:AuxThread", Section
 * 3.3), the many-ciphertext packing (Section 4.2) and version B (Algorithm
 * "alg:Softmax1B", Section 4.3), on top of the CKKS functionality the paper
 * lists in Section 2.2 ("Functionalities": KeyGen, Enc, Dec, Add, Mult, Rot)
 * plus bootstrapping (Section 2.2, "Levels").
 *
 * Conventions for every entry point
 *  - Return value: HS_OK (0) or a negative hs_status; the message of the
 *    last failure on the calling thread is returned by hs_last_error().
 *    Nothing throws across this interface.  On failure, output handles are
 *    set to NULL and caller buffers are left in an unspecified state.
 *  - Handles (hs_ctx, hs_ct) are created by the library and released with
 *    the matching destroy call.  Input handles are borrowed; every hs_ct**
 *    output is a new handle owned by the caller.
 *  - Host arrays are caller-allocated and only read or written during the
 *    call.  Device memory is owned by the context (its own caching pool).
 *  - A context is bound to one device and one HIP stream and is not
 *    thread-safe: calls on one context must not overlap.
 *  - Slots: a ciphertext holds N/2 complex slots; slot j is the evaluation
 *    of the message at zeta^(5^j mod 2N), zeta = exp(i pi / N).  Rotation by
 *    r maps slot j to slot j - r (left rotation, Galois element 5^r mod 2N).
 *  - Levels: level l means the primes q_0..q_l; multiplication lowers the
 *    level by one (Section 2.2, "Levels").  Ciphertext residues are stored
 *    in the negacyclic NTT domain, limb-major: [component][l+1][N] uint64.
 */
#ifndef HS_H
#define HS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int hs_status;
#define HS_OK 0
#define HS_E_ARG (-1)      /* bad argument (null pointer, size, index)        */
#define HS_E_PARAM (-2)    /* unsupported or inconsistent parameter set        */
#define HS_E_LEVEL (-3)    /* level exhausted or operands at unusable levels   */
#define HS_E_SCALE (-4)    /* operands with different scales                   */
#define HS_E_KEY (-5)      /* required key (relinearisation / Galois) missing  */
#define HS_E_OOM (-6)      /* device allocation failed                         */
#define HS_E_DEVICE (-7)   /* HIP runtime error                                */
#define HS_E_RANGE (-8)    /* input outside the documented range               */
#define HS_E_STATE (-9)    /* call out of order (e.g. no keys yet)             */

typedef struct hs_ctx hs_ctx;
typedef struct hs_ct hs_ct;
typedef struct hs_softmax_plan hs_softmax_plan;

/* Parameter set.  Primes are found by the rule: for a bit size b the
 * candidates are 2^b + 1 + j 2N for j = 1, -1, 2, -2, ...; the chain takes,
 * in the order q_0..q_{n_q-1} then p_0..p_{n_p-1}, the next unused prime of
 * its size.  Key-switching digits are consecutive blocks of `digit` Q primes;
 * a parameter set with a digit product above P / 2^20 (P = prod p_k) is
 * rejected with HS_E_PARAM.  The bootstrapping fields are ignored when boot_cts_levels is
 * 0; otherwise the top boot_cts_levels + boot_evalmod_levels +
 * boot_stc_levels Q primes are reserved for bootstrapping and user_top must
 * equal n_q - 1 minus that count. */
typedef struct hs_params {
    int log_n;            /* ring degree N = 2^log_n, 3 <= log_n <= 17        */
    int n_q;              /* number of Q primes                                */
    const int* q_bits;    /* [n_q] target bit sizes (32..61; HS_E_PARAM else)  */
    int n_p;              /* number of special primes                          */
    const int* p_bits;    /* [n_p] (32..61)                                    */
    int digit;            /* primes per key-switching digit                    */
    int hamming;          /* secret Hamming weight; 0 = uniform ternary        */
    double sigma;         /* discrete Gaussian parameter of the errors         */
    int log_scale;        /* default scale 2^log_scale                         */
    int user_top;         /* highest level handed to users                     */
    int boot_cts_levels;  /* bootstrapping: coefficient-to-slot levels         */
    int boot_evalmod_levels;
    int boot_stc_levels;
    int boot_K;           /* bound on |I| in the modular reduction             */
    int boot_double_angle;/* number of double-angle steps                      */
    int boot_cos_degree;  /* degree of the cosine approximation                */
    int boot_log_scale;   /* internal scale of the modular reduction           */
} hs_params;

typedef struct hs_ctx_info {
    int log_n, n, slots, n_q, n_p, top_level, user_top, dnum, digit, has_boot;
} hs_ctx_info;

/* Library version string (static storage). */
const char* hs_version(void);
/* Message of the last failure on this thread (static thread-local storage). */
const char* hs_last_error(void);

/* Device memory callbacks of a context.  alloc returns `bytes` of device
 * memory on the context's device usable in stream order on `hip_stream` (the
 * context's stream), or NULL when none is available (the call that needed it
 * then fails with HS_E_OOM); free returns a block with the size it was
 * allocated with.  The Python binding passes torch's caching allocator. */
typedef void* (*hs_alloc_fn)(size_t bytes, void* hip_stream, void* user);
typedef void (*hs_free_fn)(void* ptr, size_t bytes, void* user);

/* Create a context on HIP device `device`, issuing all work on `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  Builds the NTT tables,
 * base-conversion constants and encoding twiddles.  Every device allocation
 * of the context (tables, keys, ciphertexts, the arena's chunks, the arenas
 * of its captured schedules) goes through alloc_fn / free_fn with `user`
 * (both or neither: HS_E_ARG); without them, hipMalloc / hipFree.  The
 * callbacks must stay valid until hs_ctx_destroy, which returns every block
 * (after waiting for the stream), as does a failed creation.  Not from the
 * callbacks: the autotuner's timing buffers (process-wide) and the fixed
 * scratch of hs_mult_relin_noalloc.  HS_E_OOM when a callback returns NULL
 * during creation. */
hs_status hs_ctx_create_ex(const hs_params* p, int device, void* hip_stream, hs_alloc_fn alloc_fn,
                           hs_free_fn free_fn, void* user, hs_ctx** out);
/* A context on another HIP stream (hip_stream) that shares src's keys and
 * device tables instead of holding its own copies (the serving loop's
 * workers: one key set in HBM for all of them).  Same parameters, device and
 * allocator callbacks as src; it computes the same words as src.  Keys it
 * needs that src lacks are generated into its own memory.  src must have its
 * keys (HS_E_STATE) and must not itself be a clone (HS_E_ARG).  Destroying
 * src while clones live releases the handle at once and src's device memory
 * when its last clone is destroyed.  hs_keygen is refused (HS_E_STATE) on a
 * clone and on a context with live clones.  Each context is still
 * single-stream and not thread-safe; a context and its clones may be used
 * from different threads at once (they share only read-only key memory). */
hs_status hs_ctx_clone(hs_ctx* src, void* hip_stream, hs_ctx** out);
/* hs_ctx_create_ex without callbacks (hipMalloc / hipFree). */
hs_status hs_ctx_create(const hs_params* p, int device, void* hip_stream, hs_ctx** out);
void hs_ctx_destroy(hs_ctx* ctx);
hs_status hs_ctx_get_info(const hs_ctx* ctx, hs_ctx_info* info);
/* The primes, Q then P: writes min(cap, n_q + n_p) values, *n = n_q + n_p. */
hs_status hs_ctx_primes(const hs_ctx* ctx, uint64_t* out, size_t cap, size_t* n);
/* Block until all work issued on the context's stream has finished. */
hs_status hs_sync(hs_ctx* ctx);
/* A new HIP stream (default priority, non-blocking) on `device`, for a
 * context of its own (contexts on different streams overlap on the GPU);
 * destroy it after its contexts. */
hs_status hs_stream_create(int device, void** stream);
hs_status hs_stream_destroy(void* stream);
/* Device memory of the context's arena: bytes held by live objects (keys,
 * tables, ciphertexts) and bytes reserved from the device (8 GiB chunks).
 * Not counted: tables the context keeps outside the arena until it is
 * destroyed (conversion constants, bootstrap plaintexts, and the masked
 * normalisation plaintexts of the Softmax schedules it has run, at most
 * 8 GiB, reused by later calls of the same shape). */
hs_status hs_ctx_memory(const hs_ctx* ctx, size_t* in_use, size_t* reserved);
/* Return the arena's wholly unused chunks to the device (e.g. after a large
 * batch, so another context on the same GPU can use the memory); waits for
 * the context's stream first.  Writes the bytes released to *released (may
 * be NULL). */
hs_status hs_ctx_trim(hs_ctx* ctx, size_t* released);

/* KeyGen (Section 2.2): secret, public and relinearisation keys from one
 * 64-bit seed.  Every draw is Philox4x32-10 (Salmon et al., SC11) with
 * key = seed and counter = (coefficient index, 64-bit domain tag).  Replaces
 * every key of the context (rotation keys included).  HS_E_STATE while a
 * captured Softmax schedule (hs_softmax_plan_create) of this context is
 * alive: its graph holds the device addresses of the current keys, so
 * destroy the plans first. */
hs_status hs_keygen(hs_ctx* ctx, uint64_t seed);
/* Rotation keys for the given left-rotation steps (any sign, modulo N/2),
 * and the conjugation key when conj != 0. */
hs_status hs_add_rotation_keys(hs_ctx* ctx, const int32_t* steps, size_t n_steps, int conj);
/* Key material export for testing: key id 0 = relinearisation, otherwise a
 * Galois element.  Layout [dnum][2 (b, a)][n_q + n_p][N], NTT domain, in the
 * specified form (the device copy keeps its Q rows multiplied by P^-1 mod q_i,
 * which lets ModDown skip a product; the export multiplies them back). */
hs_status hs_key_export(hs_ctx* ctx, int key_id, uint64_t* out, size_t cap, size_t* used);
/* Secret coefficients (int64, N values) and public key ([2][n_q][N]); for
 * the client side and for tests. */
hs_status hs_secret_export(hs_ctx* ctx, int64_t* out, size_t n);
hs_status hs_pk_export(hs_ctx* ctx, uint64_t* out, size_t cap, size_t* used);

/* Encode N/2 complex slots (im may be NULL) at `scale` into NTT-domain
 * residues of q_0..q_level, written to out[(level+1) * N]. */
hs_status hs_encode(hs_ctx* ctx, const double* re, const double* im, size_t n_slots, int level, double scale,
                    uint64_t* out);
/* Enc (Section 2.2) of the encoding of the slots, at `level` and `scale`;
 * randomness from `seed`. */
hs_status hs_encode_encrypt(hs_ctx* ctx, const double* re, const double* im, size_t n_slots, int level,
                            double scale, uint64_t seed, hs_ct** out);
/* Enc of given NTT-domain plaintext residues ((level+1) * N values). */
hs_status hs_encrypt_rows(hs_ctx* ctx, const uint64_t* pt, int level, double scale, uint64_t seed, hs_ct** out);
/* Dec (Section 2.2) followed by decoding to N/2 slots (im may be NULL). */
hs_status hs_decrypt_decode(hs_ctx* ctx, const hs_ct* ct, double* re, double* im, size_t n_slots);

/* Ciphertext transport: words = ncomp * (level+1) * N residues. */
hs_status hs_ct_export(hs_ctx* ctx, const hs_ct* ct, uint64_t* words, size_t cap, size_t* used);
hs_status hs_ct_import(hs_ctx* ctx, const uint64_t* words, int level, int ncomp, double scale, hs_ct** out);
hs_status hs_ct_info(const hs_ct* ct, int* level, int* ncomp, double* scale);
hs_status hs_ct_set_scale(hs_ct* ct, double scale);
void hs_ct_destroy(hs_ct* ct);

/* Add (Section 2.2): operands at the same level and scale. */
hs_status hs_add(hs_ctx* ctx, const hs_ct* a, const hs_ct* b, hs_ct** out);
hs_status hs_sub(hs_ctx* ctx, const hs_ct* a, const hs_ct* b, hs_ct** out);
/* Tensor product (degree-2 result, no key switching). */
hs_status hs_tensor(hs_ctx* ctx, const hs_ct* a, const hs_ct* b, hs_ct** out);
/* Relinearisation of a degree-2 ciphertext (hybrid key switching). */
hs_status hs_relinearize(hs_ctx* ctx, const hs_ct* d, hs_ct** out);
/* Rescale: divide by q_level with centred rounding; level - 1. */
hs_status hs_rescale(hs_ctx* ctx, const hs_ct* a, hs_ct** out);
/* Mult (Section 2.2): tensor, relinearise and, if rescale != 0, rescale;
 * operands at different levels are first brought to the lower one. */
hs_status hs_mult_relin(hs_ctx* ctx, const hs_ct* a, const hs_ct* b, int rescale, hs_ct** out);
/* Allocation-free Mult, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the product of hs_mult_relin on raw device buffers, with every
 * intermediate in a fixed scratch array of 96 MiB per device, held by the
 * library from its first context on that device until the process ends.
 * a, b: device pointers to two degree-1 ciphertexts at `level`, each
 * [2][level+1][N] uint64 residues (NTT domain; the layout hs_ct_export
 * writes), scales scale_a and scale_b.  out: device pointer receiving
 * [2][level'+1][N] with level' = level - (rescale != 0); it must not overlap
 * a or b.  All three 256-byte aligned; they stay owned by the caller, and
 * the work is issued on the context's stream (asynchronous: synchronise
 * before reading out).  *out_scale (may be NULL) receives the output scale.
 * The words equal those of hs_mult_relin(a, b, rescale).  The call makes no
 * hipMalloc / hipFree and tunes nothing.
 * Errors: HS_E_ARG for null or misaligned pointers, overlap, non-positive
 * scales, or a level whose intermediates exceed the scratch (the message
 * gives the need; at N = 2^16 with 9 special primes and 8-prime digits,
 * levels up to 13 fit, every user level of that chain); HS_E_LEVEL for a level outside 0..top (or 0 with
 * rescale); HS_E_KEY without the relinearisation key; HS_E_STATE while the
 * launch profiler is on, or before the key-switching tables of this level
 * exist (they are built by the first key switch at that level, e.g. one
 * hs_mult_relin); HS_E_DEVICE if the scratch array's device address could
 * not be looked up.  Every call on one device shares that device's array and
 * leaves its contents behind: calls that overlap on one GPU (two host
 * threads, or contexts on different streams) race and must be serialised by
 * the caller. */
hs_status hs_mult_relin_noalloc(hs_ctx* ctx, const uint64_t* a, const uint64_t* b, int level, double scale_a,
                                double scale_b, int rescale, uint64_t* out, double* out_scale);
/* Rot (Section 2.2): left rotation of the slots by r (needs its key). */
hs_status hs_rotate(hs_ctx* ctx, const hs_ct* a, int32_t r, hs_ct** out);
/* Rot by several offsets of one ciphertext sharing one ModUp (hoisting; the
 * linear transforms of the bootstrap, Section 5.1, use it): out[i] decrypts
 * to Rot(a, rots[i]).  The words differ from hs_rotate's (another valid lift
 * of the rotated digits).  1 <= n <= 32, no rots[i] a multiple of the slot
 * count (HS_E_ARG), every key present (HS_E_KEY); writes n new handles. */
hs_status hs_rotate_hoisted(hs_ctx* ctx, const hs_ct* a, const int32_t* rots, size_t n, hs_ct** out);
/* Rot of n ciphertexts of one level and scale, a[i] by rots[i], as one batched
 * key switch (one ModUp, inner product with a key per ciphertext, ModDown);
 * out[i] equals hs_rotate(a[i], rots[i]) word for word.  1 <= n <= 32;
 * errors as hs_rotate_hoisted, HS_E_LEVEL / HS_E_SCALE for mixed inputs. */
hs_status hs_rotate_batch(hs_ctx* ctx, const hs_ct* const* a, const int32_t* rots, size_t n, hs_ct** out);
/* Complex conjugation of every slot (needs the conjugation key). */
hs_status hs_conjugate(hs_ctx* ctx, const hs_ct* a, hs_ct** out);
/* Multiply by NTT-domain plaintext residues pt[(a.level+1) * N] whose scale
 * is pt_scale; rescale if rescale != 0. */
hs_status hs_mul_plain_rows(hs_ctx* ctx, const hs_ct* a, const uint64_t* pt, double pt_scale, int rescale,
                            hs_ct** out);
/* Multiply by the signed integer k (no level consumed, scale unchanged). */
hs_status hs_mul_int(hs_ctx* ctx, const hs_ct* a, int64_t k, hs_ct** out);
/* Add the constant v to every slot (adds rint(v * scale) to the message). */
hs_status hs_add_const(hs_ctx* ctx, const hs_ct* a, double v, hs_ct** out);
/* Keep q_0..q_level (level <= the input's). */
hs_status hs_mod_drop(hs_ctx* ctx, const hs_ct* a, int level, hs_ct** out);
/* Lift a level-0 ciphertext to q_0..q_level with centred residues. */
hs_status hs_mod_raise(hs_ctx* ctx, const hs_ct* a, int level, hs_ct** out);
/* Multiply by the monomial X^k (k modulo 2N). */
hs_status hs_mul_monomial(hs_ctx* ctx, const hs_ct* a, int k, hs_ct** out);

/* ---------------------------------------------------------------- Softmax
 * Options of hs_softmax.  variant 0 = Algorithm SM (Section 3.2, with the
 * auxiliary thread of Section 3.3 and the packing of Section 4); variant 1 =
 * SM version B (Algorithm "alg:Softmax1B", Section 4.3).  k = 0 selects
 * k = ceil(log2 M - log2 ln n) (Theorem "th:prec_softmax"). */
typedef struct hs_softmax_opts {
    int variant;
    int k;                /* 0 = the Theorem's k (+1 from n = 4096)           */
    int exp_degree;       /* degree of the exp approximation, 2^t - 1; 0 = 15 */
    int inv_degree_first; /* degree of the first normalisation polynomial     */
    int inv_degree_mid;   /* intermediate iterations                          */
    int inv_degree_last;  /* last iteration; 0 for any of the three: 2^d - 1  */
                          /* by dimension n: up to 256 the paper's depths at  */
                          /* n = 256 (Section 5, auxiliary-thread level       */
                          /* table: 6, 5, 7); n <= 1024: 6, 6, 8; larger:     */
                          /* 7, 7, 8                                          */
    double alpha;         /* reserved (0)                                     */
    int power;            /* t of the normalize-and-t-th-power variant (the   */
                          /* appendix on other normalisations: lambda =      */
                          /* (sum y^t)^(-1/t), y <- (lambda y)^t, exp of     */
                          /* x / t^k with M / t^k ~ ln n); 0 or 2 = squares; */
                          /* 3 or 4 with variant 0 only (HS_E_PARAM else)    */
    int debug_stop;       /* tests: >= 0 returns y after that iteration
                             (0 = after the exponential); -1 = off          */
    int newton_steps;     /* > 0: each inverse square root by that many       */
                          /* Newton steps (Appendix A) from the normalisation */
                          /* polynomial as first guess (the guess             */
                          /* bootstrapped first when its depth and the steps  */
                          /* exceed the levels a bootstrap restores); version */
                          /* B takes one in its last step only; squares only  */
                          /* (HS_E_PARAM else); 0 = by dimension: none up to  */
                          /* n = 2048, 2 above; -1 = none                     */
    int mask_mode;        /* 0: mask = indicator of slots [0, L); 1: the      */
                          /* averaging mask (m / n on every slot, no          */
                          /* plaintext; bootstraps of the factors unmasked)   */
    int approx;           /* normalisation polynomials: 0 = the weighted      */
                          /* minimax approximants (Section 5.1; smallest max  */
                          /* relative error on the interval), 1 = Chebyshev   */
                          /* interpolants (larger worst case, smaller error   */
                          /* away from the interval's lower end)              */
    int merge;            /* hs_softmax_jobs with version B: 1 = the jobs'    */
                          /* auxiliary ciphertexts packed (Section 4.2: one   */
                          /* auxiliary ciphertext carries the sums of many    */
                          /* Softmax), n / m jobs per ciphertext, job         */
                          /* g n/m + b's sums on slots [bL, (b+1)L) of the    */
                          /* g-th, so each sum, polynomial and bootstrap of   */
                          /* the auxiliary thread covers n / m jobs at once;  */
                          /* each job's factor is taken back by a 0/1         */
                          /* plaintext product (one level) before its         */
                          /* broadcast.  Needs njobs <= n / m or a multiple   */
                          /* of it, squares with the indicator mask and no    */
                          /* Newton steps (HS_E_PARAM else).  A job's result  */
                          /* then depends on the others through the shared    */
                          /* bootstraps' noise: equal to its result alone     */
                          /* within the precision, not word for word.         */
                          /* 0 = separate auxiliary ciphertexts (one batch)   */
} hs_softmax_opts;

/* Softmax (Eq. "eq:smdef") of the L = m (N/2) / n vectors of dimension n
 * packed in the m ciphertexts in[0..m) (layout of hs_pack_softmax), all at
 * the same level and scale, inputs in [-M, 0] (the paper's assumption of
 * Section 3.1; values outside give unspecified results).  For the first step
 * to cost no level, encrypt the inputs at scale D = 2^(log_scale + 1) / M;
 * inputs at level l >= 1 and scale D q_l take one rescale first, which
 * divides their encryption noise by q_l (at scale D that noise limits the
 * output to about 16.5 bits at N = 2^16: an absolute logit error becomes a
 * relative output error); other scales take one constant product.
 * Writes m new handles to out[0..m).  A dimension n that is not a power of
 * two is packed (hs_pack_softmax) as the next power of two n2, and the
 * exponentials of the extra coordinates are removed by one plaintext mask
 * product (one level) before the first normalisation, so every sum runs over
 * the n real coordinates (the rounded-up log n of the auxiliary thread's
 * rotation count).  Needs m | n2, n2 <= N/2 (HS_E_ARG otherwise), enough
 * levels or bootstrapping parameters (HS_E_LEVEL).  Rotation keys for strides +-L 2^t are generated
 * on first use. */
hs_status hs_softmax(hs_ctx* ctx, hs_ct* const* in, size_t m, uint32_t n, double M, const hs_softmax_opts* opts,
                     hs_ct** out);
/* Several independent Softmax jobs of one shape in lockstep (batched
 * many-Softmax, Section 4.2, applied to njobs jobs at once): in[0..m) holds
 * njobs consecutive jobs of m / njobs ciphertexts each, every job packed as
 * hs_pack_softmax packs it, all with the same n, M, level and scale.  Every
 * launch of the main thread covers all m ciphertexts; the njobs auxiliary
 * ciphertexts (Algorithm "alg:AuxThread") form one batch, so each of their
 * key switches and bootstraps reads its keys once for all jobs.  Every
 * operation acts per ciphertext, so job j's outputs are bit for bit those of
 * hs_softmax on job j alone.  Writes m new handles, job by job.  Errors as
 * hs_softmax; HS_E_ARG when njobs does not divide m. */
hs_status hs_softmax_jobs(hs_ctx* ctx, hs_ct* const* in, size_t m, size_t njobs, uint32_t n, double M,
                          const hs_softmax_opts* opts, hs_ct** out);
/* Statistics of the last hs_softmax(_jobs) call: [k, bootstraps (auxiliary
 * and main ciphertexts refreshed), levels_left, milliseconds]; writes
 * min(n, 4) values. */
hs_status hs_softmax_stats(hs_ctx* ctx, double* out, size_t n);

/* Captured Softmax schedule (a HIP graph).  The schedule of hs_softmax_jobs
 * (Algorithms SM / SM-B with the many-ciphertext packing of Section 4.2) is
 * fixed by the ciphertext count, job count, n, M, the options and the input
 * level and scale, so it is recorded once and replayed.
 * hs_softmax_plan_create: `in` (m handles of one ciphertext each, one level,
 * one scale) is both the shape template and the input of one eager warm-up
 * run, which builds every table and key the schedule needs; the schedule is
 * then captured on a stream of the plan's own.  The plan owns a private
 * device arena (its input, intermediate and output buffers keep their
 * addresses across replays); it borrows the context, which must outlive it.
 * Errors as hs_softmax_jobs; HS_E_STATE when the launch profiler is enabled
 * or another capture is in progress.
 * hs_softmax_plan_run: copies the m inputs (same level, size and scale as
 * the template, else HS_E_LEVEL / HS_E_SCALE) into the plan, replays the
 * graph and writes m new output handles (results bit for bit those of
 * hs_softmax_jobs on the same inputs).  Synchronous; updates
 * hs_softmax_stats.  Replays of one plan must not overlap (one host thread).
 * hs_softmax_plan_info: graph node count and arena bytes (either may be NULL).
 * hs_softmax_plan_destroy: waits for the plan's stream and frees everything.
 * While a plan is alive, hs_keygen on its context returns HS_E_STATE (the
 * graph replays with the keys it was recorded with). */
hs_status hs_softmax_plan_create(hs_ctx* ctx, hs_ct* const* in, size_t m, size_t njobs, uint32_t n, double M,
                                 const hs_softmax_opts* opts, hs_softmax_plan** out);
hs_status hs_softmax_plan_run(hs_softmax_plan* plan, hs_ct* const* in, size_t m, hs_ct** out);
hs_status hs_softmax_plan_info(const hs_softmax_plan* plan, size_t* nodes, size_t* arena_bytes);
void hs_softmax_plan_destroy(hs_softmax_plan* plan);

/* Autotuner (not in the paper: an implementation choice).  Some operations
 * have interchangeable kernels that give identical results: the base
 * conversion of hybrid key switching (exact 128-bit VALU sums with the
 * targets on 1, 2 or 4 threads per coefficient, or int8 byte planes on the
 * matrix cores) and the N = 2^16 NTT (row order, launch batching over row
 * groups).  While tuning is enabled (or HS_TUNE=1 in the
 * environment), the first launch of each shape (N, sources, targets, row
 * groups rounded up to a power of two) times every candidate on scratch
 * data, rejects any whose output differs from the default kernel's, and keeps
 * the fastest for the process; never during graph capture.  Decisions are
 * process-wide and apply to every context.
 * hs_tune_enable: on != 0 enables tuning of shapes not yet decided.
 * hs_tune_clear: forgets every decision (the default kernels again).
 * hs_tune_report: the decisions as text, one JSON object per line
 * ({"key", "choice", "us": candidate times in microseconds, < 0 rejected});
 * writes min(cap, size) bytes NUL-terminated and the full size + 1 to *used.
 * hs_tune_save / hs_tune_load: write / read that text to / from a file;
 * loaded decisions replace tuned ones of the same key (HS_E_ARG when the
 * file cannot be opened). */
hs_status hs_tune_enable(int on);
hs_status hs_tune_clear(void);
hs_status hs_tune_report(char* buf, size_t cap, size_t* used);
hs_status hs_tune_save(const char* path);
hs_status hs_tune_load(const char* path, int* entries);

/* Packing of Section 4 (host only).  logits: [L][n] row-major, L n2 =
 * m (N/2) with n2 the power of two at or above n; out: [m][slots] with
 * ciphertext j holding coordinate j (n2/m) + c of Softmax l in slot c L + l
 * (coordinates n..n2-1, if any, set to -M).  Checks every logit is in
 * [-M, 0] (HS_E_RANGE otherwise). */
hs_status hs_pack_softmax(const double* logits, size_t L, uint32_t n, size_t slots, double M, double* out,
                          size_t* m_out);
/* Inverse of hs_pack_softmax: slots [m][slots] -> out [L][n] (padding
 * coordinates dropped). */
hs_status hs_unpack_softmax(const double* slots_in, size_t m, uint32_t n, size_t slots, double* out);

/* Bootstrapping: refresh a ciphertext (any level) to the top user level
 * (CoeffToSlot, EvalMod, SlotToCoeff).  HS_E_PARAM without bootstrapping
 * parameters; needs the conjugation and linear-transform rotation keys,
 * generated on first use. */
hs_status hs_bootstrap(hs_ctx* ctx, const hs_ct* a, hs_ct** out);

/* Launch profiling with HIP events on the context's stream.  When enabled,
 * every launch of the NTT, key-switching inner product, base conversion,
 * tensor, elementwise, permutation and lift kernels records an event pair and
 * its algorithmic bytes (compulsory reads and writes).  hs_prof_collect
 * waits for the recorded events and writes, for kinds 0..7 (NTT, KEYIP,
 * CONV, TENSOR, EW, PERM, LIFT, OTHER), [launches, milliseconds, bytes]
 * (n >= 24), then clears the record. */
hs_status hs_prof_enable(hs_ctx* ctx, int on);
hs_status hs_prof_collect(hs_ctx* ctx, double* out, size_t n);

/* Homomorphic operations issued by the context since the last clear (not an
 * operation of the paper: an account of the schedule for cost models of other
 * implementations of it), by kind and input level, in ciphertext equivalents
 * (one degree-1 ciphertext = 1): kind 0 key switches (relinearisations,
 * rotations, conjugations), 1 tensor products (squares included), 2 rescales,
 * 3 plaintext or constant products, 4 additions.  Writes min(n, 5 * 64)
 * values out[kind * 64 + level] (out may be NULL); clears the counts when
 * clear != 0.  Graph replays (hs_softmax_plan_run) are not counted. */
hs_status hs_op_counts(hs_ctx* ctx, double* out, size_t n, int clear);

/* Intermediate ciphertexts of hs_bootstrap, for tests: stage 1 = after
 * ModRaise (declared scale 2 q0 (K+1) N/2), 2 = after CoeffToSlot, 3 = real
 * part u after the conjugation split, 4 = real-part half of
 * z = exp(2 pi i (K+1) u / 2^r) after the two Chebyshev polynomials,
 * 5 / 6 = real / imaginary half of z after the r squarings, 7 = input of
 * SlotToCoeff (2 (8 sin x - sin 2x) per coefficient, recombined), 8 / 9 =
 * after its first / second level. */
hs_status hs_dbg_bootstrap_stage(hs_ctx* ctx, const hs_ct* a, int stage, hs_ct** out);

/* Device time of the NTT kernels (not an operation of the paper; for kernel
 * measurements): `groups` groups of level+1 rows of pseudo-random residues
 * (the layout of one ciphertext component per group, row i modulo q_i) are
 * transformed `reps` times (forward, or inverse when inverse != 0) on the
 * context's stream; *us receives the average microseconds per transform
 * launch over all groups.  HS_E_ARG for groups outside 1..4096 or reps
 * outside 1..1000, HS_E_LEVEL for a level outside 0..top. */
hs_status hs_dbg_ntt_time(hs_ctx* ctx, int groups, int level, int reps, int inverse, double* us);

/* Raw negacyclic NTT (forward or inverse) of `nrows` rows of N residues
 * modulo prime index `prime` (host buffer, in place); for parity tests. */
hs_status hs_dbg_ntt(hs_ctx* ctx, int prime, uint64_t* rows, size_t nrows, int inverse);

/* Raw ring operations on host rows, for parity tests of the primitives
 * beneath key switching and rescaling (the paper relies on them through its
 * CKKS library: Section 2.2, "Functionalities" and "Levels"; it specifies
 * none of their internals).  Rows are N residues each, NTT domain unless
 * stated, rows of prime q_i at index i; `in` holds in_words words and out
 * receives *out_words words (out may be NULL or out_cap 0 to query the
 * size).  HS_E_ARG when in_words does not match the operation, HS_E_LEVEL
 * for a level outside 0..top.
 *   HS_DBG_NTT / HS_DBG_INTT: rows q_0..q_level from coefficients / back.
 *   HS_DBG_MODUP: one polynomial at `level` (level+1 rows) -> its hybrid
 *     key-switching extension [beta][level+1+n_p][N], beta =
 *     ceil((level+1)/digit): digit j (Q rows j*digit..) lifted to every
 *     other prime of Q_level u P by the fast base conversion, NTT domain,
 *     the digit's own rows unchanged.
 *   HS_DBG_MODDOWN: one polynomial over Q_level u P ((level+1+n_p) rows,
 *     q_0..q_level then p_0..) -> (c - Conv_P->Q([c]_P)) P^-1 mod q_i
 *     (centred conversion), level+1 rows.
 *   HS_DBG_AUTO: X -> X^arg (arg an odd Galois element, modulo 2N) on
 *     level+1 rows.
 *   HS_DBG_RESCALE: (c - r) q_level^-1 with r the centred residue of c mod
 *     q_level; level+1 rows in, level rows out (level >= 1).
 *   HS_DBG_TENSOR: two degree-1 ciphertexts (a0, a1, b0, b1: 4 (level+1)
 *     rows) -> (a0 b0, a0 b1 + a1 b0, a1 b1): 3 (level+1) rows. */
#define HS_DBG_NTT 0
#define HS_DBG_INTT 1
#define HS_DBG_MODUP 2
#define HS_DBG_MODDOWN 3
#define HS_DBG_AUTO 4
#define HS_DBG_RESCALE 5
#define HS_DBG_TENSOR 6
hs_status hs_dbg_ring(hs_ctx* ctx, int op, int level, int arg, const uint64_t* in, size_t in_words,
                      uint64_t* out, size_t out_cap, size_t* out_words);

/* Measured throughput of v_mad_u64_u32 (32 x 32 + 64 -> 64 bit), the
 * instruction the 64-bit modular products are built from, in 10^12 lane
 * operations per second (eight independent chains per lane, about 1 ms on
 * the context's device and stream).  HS_E_DEVICE if the probe fails. */
hs_status hs_dbg_mul_rate(hs_ctx* ctx, double* tops);

/* Host only: the coefficients c[0..degree] (Chebyshev basis of [a, b]) of the
 * normalisation polynomial the Softmax evaluates for s^-e on [a, b]: the
 * weighted minimax approximant minimising max |P(s) s^e - 1| (Section 5.1,
 * "Designing auxiliary functions"), as the Remez exchange on the fixed grid
 * u_i = -cos(pi i / (G - 1)), G = 16 (degree + 1) + 1, specified in
 * csrc/poly.h.  0 < a < b, e > 0, degree 0..1023 (HS_E_ARG otherwise). */
hs_status hs_dbg_minimax(double a, double b, int degree, double e, double* c);

#ifdef __cplusplus
}
#endif
#endif /* HS_H */
