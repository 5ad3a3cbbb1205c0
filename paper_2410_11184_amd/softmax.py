"""Client-side helpers around ``hs_softmax``: pack logits (Section 4
layout), encrypt them at a scale that makes the first step a rescale or
nothing, run the encrypted Softmax on the GPU, decrypt and unpack.  All arithmetic runs in
``libhs.so``."""
import numpy as np

from . import hs


def encrypt_logits(ctx, logits, M, seed, level=None, headroom=True):
    """Pack (L, n) logits into m ciphertexts.  With a level above the top
    user level (rings with bootstrapping) and headroom set, they are encrypted
    there at scale (2 Delta / M) q_l: the Softmax's first step is then one
    rescale, which divides the encryption noise by q_l (at scale 2 Delta / M
    that noise bounds the output's precision near 16.5 bits at N = 2^16).
    Otherwise at the top user level (or `level`) and scale 2 Delta / M."""
    packed = hs.pack_softmax(logits, ctx.slots, M)
    scale = ctx.delta * 2.0 / M
    if level is None:
        level = ctx.user_top
        if headroom and ctx.L > ctx.user_top:
            level = ctx.user_top + 1
            scale *= float(ctx.primes()[level])
    return [ctx.encrypt(packed[j], level, scale, seed + j) for j in range(packed.shape[0])]


def decrypt_outputs(ctx, cts, n):
    slots = np.stack([ctx.decrypt(c).real for c in cts])
    return hs.unpack_softmax(slots, n)


def softmax_encrypted(ctx, logits, M, variant="SM", seed=1, k=0, exp_degree=0, inv_degrees=(0, 0, 0)):
    """Encrypt, evaluate Softmax homomorphically, decrypt.  Returns (L, n)."""
    logits = np.asarray(logits, dtype=np.float64)
    n = logits.shape[1]
    cts = encrypt_logits(ctx, logits, M, seed)
    out = ctx.softmax(cts, n, M, variant=1 if variant in ("B", "SMB", 1) else 0, k=k,
                      exp_degree=exp_degree, inv_degrees=inv_degrees)
    return decrypt_outputs(ctx, out, n)


def softmax_jobs_encrypted(ctx, logits_list, M, variant="B", seed=1, k=0, exp_degree=0, inv_degrees=(0, 0, 0)):
    """Several independent Softmax jobs of one shape (same n and vector count)
    evaluated in lockstep by hs_softmax_jobs.  Returns one (L, n) array per job."""
    logits_list = [np.asarray(x, dtype=np.float64) for x in logits_list]
    n = logits_list[0].shape[1]
    cts, counts = [], []
    for j, x in enumerate(logits_list):
        if x.shape != logits_list[0].shape:
            raise ValueError("jobs of one lockstep group must share their shape")
        c = encrypt_logits(ctx, x, M, seed + 1000 * j)
        cts += c
        counts.append(len(c))
    out = ctx.softmax(cts, n, M, variant=1 if variant in ("B", "SMB", 1) else 0, k=k, exp_degree=exp_degree,
                      inv_degrees=inv_degrees, jobs=len(logits_list))
    res, o = [], 0
    for cnt in counts:
        res.append(decrypt_outputs(ctx, out[o:o + cnt], n))
        o += cnt
    return res


def softmax_groups(runs):
    """Softmax calls of different shapes at once (an uneven batch): `runs` is
    a list of (context, ciphertexts, n, M, options), each context on a HIP
    stream of its own (a context and its clones, hs_ctx_clone, share one key
    set), each call's ciphertexts encrypted by its context.  Every call runs
    in a host thread of its own, so the GPU overlaps the groups' launches
    (the small launches of one group's single-ciphertext auxiliary thread
    fill what another group leaves idle); a call with options jobs=J runs J
    same-shape jobs in lockstep.  Every operation acts per ciphertext and per
    context, so each call's outputs are the words it gives alone.  Returns
    [(outputs, stats)] in order; the first error raised by a call is raised
    here after every thread has ended."""
    import threading
    res = [None] * len(runs)
    errs = [None] * len(runs)

    def work(i):
        ctx, cts, n, M, kw = runs[i]
        try:
            out = ctx.softmax(cts, n, M, **kw)
            ctx.sync()
            res[i] = (out, ctx.softmax_stats())
        except BaseException as e:   # re-raised in the caller's thread
            errs[i] = e

    threads = [threading.Thread(target=work, args=(i,)) for i in range(len(runs))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    for e in errs:
        if e is not None:
            raise e
    return res
