"""Contexts that share their parent's keys (hs_ctx_clone), toy ring N = 2^12:
a clone on another stream computes the same words as its parent, holds no
copy of the parent's keys, generates keys the parent lacks into its own
memory, refuses key generation on both sides while it lives, and keeps
working after its parent's handle is destroyed."""
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
