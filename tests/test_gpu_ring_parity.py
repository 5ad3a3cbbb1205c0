"""Bit-exact parity of every ring / CKKS operation of the HIP library with
the CPU oracle, on the same seeds, through the C ABI.

Toy ring N = 2^12 with 24 + 2 primes (several NTT tiles, both digit kinds)
element by element; full-size N = 2^16 parity is in test_gpu_full_size.py.
"""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

SEED = 20240917


@pytest.fixture(scope="module")
def pair():
    from paper_2410_11184_amd import hs
    from oracle import ckks
    p = synthetic.preset("toy12")
    g = hs.Context(p)
    o = ckks.Context(**p)
    rots = [1, -3, 128, 1000]
    g.keygen(SEED, rotations=rots, conj=True)
    o.keygen(SEED, galois=[o.galois_rot(r, o.N) for r in rots] + [2 * o.N - 1])
    return g, o


def _same(gct, oct_):
    w = gct.export()
    assert w.shape[0] == len(oct_.c) and w.shape[1] == oct_.level + 1
    for k in range(len(oct_.c)):
        assert np.array_equal(w[k], oct_.c[k]), "component %d differs" % k
    assert gct.level == oct_.level


def _z(N, seed, cplx=True):
    r = np.random.default_rng(seed)
    z = r.uniform(-1, 1, N // 2)
    return z + 1j * r.uniform(-1, 1, N // 2) if cplx else z


def test_primes(pair):
    g, o = pair
    assert g.primes() == o.primes


def test_ntt_rows(pair):
    g, o = pair
    rng = np.random.default_rng(1)
    for idx in (0, 7, 23, 24, 25):
        q = o.primes[idx]
        x = rng.integers(0, q, (3, o.N), dtype=np.uint64)
        f = g.ntt(x, idx)
        for r in range(3):
            assert np.array_equal(f[r], o.ntt(x[r], idx))
        back = g.ntt(f, idx, inverse=True)
        assert np.array_equal(back, x)


def test_keys(pair):
    g, o = pair
    assert np.array_equal(g.secret(), o.s_coeff)
    pk = g.pk_export()
    assert np.array_equal(pk[0], np.stack(o.pk0)) and np.array_equal(pk[1], np.stack(o.pk1))
    for kid in [0, o.galois_rot(1, o.N), 2 * o.N - 1]:
        kg = g.key_export(kid)
        ko = o.keys[kid]
        for j in range(o.dnum):
            assert np.array_equal(kg[j, 0], np.stack(ko[j][0])), (kid, j)
            assert np.array_equal(kg[j, 1], np.stack(ko[j][1])), (kid, j)


def test_encode_and_encrypt(pair):
    g, o = pair
    z = _z(o.N, 2)
    for level, scale in [(o.L, o.delta), (5, 2.0 ** 35), (0, 2.0 ** 30)]:
        pg = g.encode(z, level, scale)
        po, _ = o.encode(z, scale, level)
        assert np.array_equal(pg, np.stack(po))
        _same(g.encrypt(z, level, scale, 77), o.encode_encrypt(z, scale, level, 77))
    # real slots, large scale (values beyond 2^63 are encoded exactly)
    zr = _z(o.N, 3, cplx=False) * 1e3
    pg = g.encode(zr, 10, 2.0 ** 58)
    po, _ = o.encode(zr, 2.0 ** 58, 10)
    assert np.array_equal(pg, np.stack(po))


@pytest.fixture(scope="module")
def cts(pair):
    g, o = pair
    za, zb = _z(o.N, 4), _z(o.N, 5)
    return (g.encrypt(za, 20, o.delta, 11), g.encrypt(zb, 20, o.delta, 12),
            o.encode_encrypt(za, o.delta, 20, 11), o.encode_encrypt(zb, o.delta, 20, 12), za, zb)


def test_add_sub(pair, cts):
    g, o = pair
    ga, gb, oa, ob, _, _ = cts
    _same(g.add(ga, gb), o.add_ct(oa, ob))
    _same(g.sub(ga, gb), o.sub_ct(oa, ob))


def test_tensor_relin_rescale_mult(pair, cts):
    g, o = pair
    ga, gb, oa, ob, za, zb = cts
    t = g.tensor(ga, gb)
    ot = o.tensor(oa, ob)
    _same(t, ot)
    r = g.relinearize(t)
    orl = o.relinearize(ot)
    _same(r, orl)
    s = g.rescale(r)
    _same(s, o.rescale(orl))
    m = g.mult(ga, gb)
    om = o.mult(oa, ob)
    _same(m, om)
    assert np.max(np.abs(g.decrypt(m) - za * zb)) < 2 ** -18
    # operands at different levels: the higher one is dropped first
    m2 = g.mult(m, ga)
    _same(m2, o.mult(om, o.mod_drop(oa, om.level)))


@pytest.mark.parametrize("r", [1, -3, 128, 1000])
def test_rotation(pair, cts, r):
    g, o = pair
    ga, _, oa, _, za, _ = cts
    out = g.rotate(ga, r)
    _same(out, o.rotate(oa, r))
    assert np.max(np.abs(g.decrypt(out) - np.roll(za, -r))) < 2 ** -18


def test_conjugate(pair, cts):
    g, o = pair
    ga, _, oa, _, za, _ = cts
    out = g.conjugate(ga)
    _same(out, o.conjugate(oa))
    assert np.max(np.abs(g.decrypt(out) - np.conj(za))) < 2 ** -18


def test_rotate_batch_matches_the_oracle(pair, cts):
    # several ciphertexts, each with its own rotation, in one key switch
    g, o = pair
    ga, gb, oa, ob, za, zb = cts
    outs = g.rotate_batch([ga, gb, ga, gb], [1, -3, 1000, 128])
    for out, (oc, r) in zip(outs, [(oa, 1), (ob, -3), (oa, 1000), (ob, 128)]):
        _same(out, o.rotate(oc, r))


def test_rotate_hoisted(pair, cts):
    # one ModUp for all rotations: the oracle's hoisted rotation word for
    # word (another valid lift than rotate()'s, with the same values)
    from paper_2410_11184_amd import hs
    g, o = pair
    ga, _, oa, _, za, _ = cts
    rots = [1, -3, 128, 1000]
    for out, oout, r in zip(g.rotate_hoisted(ga, rots), o.rotate_hoisted(oa, rots), rots):
        assert out.level == ga.level and out.scale == ga.scale
        _same(out, oout)
        assert np.max(np.abs(g.decrypt(out) - np.roll(za, -r))) < 2 ** -18
    with pytest.raises(hs.HSError) as e:
        g.rotate_hoisted(ga, [1, g.slots])
    assert e.value.name == "HS_E_ARG"
    with pytest.raises(hs.HSError) as e:
        g.rotate_hoisted(ga, [5])
    assert e.value.name == "HS_E_KEY"


def test_constants_and_plain(pair, cts):
    g, o = pair
    ga, _, oa, _, za, _ = cts
    _same(g.mul_int(ga, -7), o.mul_int(oa, -7))
    _same(g.add_const(ga, 0.3125), o.add_int(oa, int(np.rint(0.3125 * oa.scale))))
    w = _z(o.N, 9, cplx=False)
    pg = g.encode(w, 20, float(o.q[20]))
    po, _ = o.encode(w, float(o.q[20]), 20)
    _same(g.mul_plain_rows(ga, pg, float(o.q[20]), rescale=True),
          o.rescale(o.mul_plain(oa, po, float(o.q[20]))))
    _same(g.mul_monomial(ga, o.N // 2), o.mul_monomial(oa, o.N // 2))
    _same(g.mul_monomial(ga, 3 * o.N // 2 + 5), o.mul_monomial(oa, 3 * o.N // 2 + 5))


def test_mod_drop_and_raise(pair, cts):
    g, o = pair
    ga, _, oa, _, _, _ = cts
    d = g.mod_drop(ga, 0)
    od = o.mod_drop(oa, 0)
    _same(d, od)
    _same(g.mod_raise(d, 17), o.mod_raise(od, 17))


def test_import_export_roundtrip(pair, cts):
    g, o = pair
    _, _, oa, _, _, _ = cts
    ct = g.import_ct(np.stack(oa.c), oa.level, 2, oa.scale)
    _same(ct, oa)


def test_errors(pair, cts):
    from paper_2410_11184_amd import hs
    g, o = pair
    ga, gb, _, _, _, _ = cts
    with pytest.raises(hs.HSError) as e:
        g.rotate(ga, 5)               # no key for 5
    assert e.value.name == "HS_E_KEY"
    low = g.mod_drop(ga, 0)
    with pytest.raises(hs.HSError) as e:
        g.rescale(low)
    assert e.value.name == "HS_E_LEVEL"
    with pytest.raises(hs.HSError) as e:
        g.add(ga, g.mul_plain_rows(gb, g.encode(_z(o.N, 1), 20, 2.0 ** 20), 2.0 ** 20))
    assert e.value.name == "HS_E_SCALE"
