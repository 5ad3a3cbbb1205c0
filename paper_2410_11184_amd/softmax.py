"""Client-side helpers around ``hs_softmax``: pack logits (Section 4
layout), encrypt them at the scale that makes the first step free, run the
encrypted Softmax on the GPU, decrypt and unpack.  All arithmetic runs in
``libhs.so``."""
import numpy as np

from . import hs


def encrypt_logits(ctx, logits, M, seed, level=None):
    """Pack (L, n) logits into m ciphertexts at scale 2 Delta / M."""
    packed = hs.pack_softmax(logits, ctx.slots, M)
    level = ctx.user_top if level is None else level
    scale = ctx.delta * 2.0 / M
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
