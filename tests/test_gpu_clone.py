"""Contexts that share their parent's keys (hs_ctx_clone), toy ring N = 2^12:
a clone on another stream computes the same words as its parent, holds no
copy of the parent's keys, generates keys the parent lacks into its own
memory, refuses key generation on both sides while it lives, and keeps
working after its parent's handle is destroyed; an uneven batch (groups of
different shapes run at once on a context and its clone, softmax_groups)
gives each group the words it gives alone."""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

SEED = 321


def _words(ct):
    w = ct.export()
    return np.stack([w[0], w[1]])


def test_clone_shares_keys_and_computes_the_same_words():
    from paper_2410_11184_amd import hs
    p = synthetic.preset("toy12")
    parent = hs.Context(p)
    parent.keygen(SEED, rotations=[1, 4])
    used_before, _ = parent.memory()
    st = hs.stream_create(0)
    clone = parent.clone(st)
    used_clone, _ = clone.memory()
    # the relinearisation and rotation keys stay in the parent's arena
    assert used_clone < used_before / 4, (used_clone, used_before)
    rng = np.random.default_rng(3)
    z = rng.uniform(-1, 1, p["slots"])
    lv = p["user_top"]
    a = [ctx.encrypt(z, lv, parent.delta, 11) for ctx in (parent, clone)]
    b = [ctx.encrypt(z[::-1].copy(), lv, parent.delta, 12) for ctx in (parent, clone)]
    assert np.array_equal(_words(a[0]), _words(a[1]))
    prod = [ctx.mult(x, y) for ctx, x, y in zip((parent, clone), a, b)]
    assert np.array_equal(_words(prod[0]), _words(prod[1]))
    rot = [ctx.rotate(x, 4) for ctx, x in zip((parent, clone), a)]
    assert np.array_equal(_words(rot[0]), _words(rot[1]))
    # a stride the parent has no key for: the clone generates its own key,
    # the same words as the parent's once the parent adds it
    clone.add_rotation_keys([8])
    r_clone = clone.rotate(a[1], 8)
    parent.add_rotation_keys([8])
    r_parent = parent.rotate(a[0], 8)
    assert np.array_equal(_words(r_clone), _words(r_parent))
    # key generation would free keys the clone reads
    for ctx in (parent, clone):
        with pytest.raises(hs.HSError) as e:
            ctx.keygen(SEED + 1)
        assert e.value.name == "HS_E_STATE"
    # a clone of a clone is refused
    with pytest.raises(hs.HSError) as e:
        clone.clone(st)
    assert e.value.name == "HS_E_ARG"
    # the parent's handle destroyed first: its memory lives until the clone's end
    want = _words(prod[1])
    del a[0], b[0], prod[0], rot[0], r_parent
    parent.close()
    again = clone.mult(a[0], b[0])
    assert np.array_equal(_words(again), want)
    dec = clone.decrypt(again)
    assert np.max(np.abs(dec - z * z[::-1])) < 1e-6
    del a, b, prod, rot, r_clone, again
    clone.close()
    hs.stream_destroy(st)


TOY = dict(exp_degree=7, inv_degrees=(15, 15, 31))


def test_uneven_groups_at_once_equal_each_alone():
    from paper_2410_11184_amd import hs
    from paper_2410_11184_amd.softmax import encrypt_logits, softmax_groups
    from oracle import softmax as S
    p = synthetic.preset("toy12")
    parent = hs.Context(p)
    parent.keygen(SEED + 7)
    st = hs.stream_create(0)
    clone = parent.clone(st)
    # group A: 3 jobs of dimension 16 (version B, 2 ciphertexts each, lockstep);
    # group B: one job of dimension 8 (Algorithm SM, 1 ciphertext)
    xa = [synthetic.logits_uniform(2 * p["slots"] // 16, 16, 8.0, seed=820 + j) for j in range(3)]
    xb = synthetic.logits_uniform(p["slots"] // 8, 8, 8.0, seed=830)
    kw_a = dict(variant=1, jobs=3, **TOY)
    kw_b = dict(variant=0, **TOY)
    ca = [c for j, x in enumerate(xa) for c in encrypt_logits(parent, x, 8.0, seed=840 + 10 * j)]
    cb = encrypt_logits(clone, xb, 8.0, seed=850)
    alone_a = [c.export() for c in parent.softmax(ca, 16, 8.0, **kw_a)]
    alone_b = [c.export() for c in clone.softmax(cb, 8, 8.0, **kw_b)]
    (out_a, st_a), (out_b, st_b) = softmax_groups([(parent, ca, 16, 8.0, kw_a), (clone, cb, 8, 8.0, kw_b)])
    for got, want in ((out_a, alone_a), (out_b, alone_b)):
        assert len(got) == len(want)
        for g, w in zip(got, want):
            e = g.export()
            assert np.array_equal(e[0], w[0]) and np.array_equal(e[1], w[1])
    ya = [S.unpack(np.stack([parent.decrypt(c).real for c in out_a[2 * j:2 * j + 2]]), 16) for j in range(3)]
    yb = S.unpack(np.stack([clone.decrypt(c).real for c in out_b]), 8)
    for x, y in zip(xa + [xb], ya + [yb]):
        assert S.precision_bits(S.softmax(x), y)["worst"] >= 12.0
    del out_a, out_b, ca, cb
    clone.close()
    parent.close()
    hs.stream_destroy(st)
