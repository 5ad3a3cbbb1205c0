"""Bit-exact parity of the raw ring primitives beneath key switching and
rescaling (hs_dbg_ring) with the CPU oracle: ModUp (fast base conversion of
every digit, NTT domain), ModDown (centred conversion from P, times P^-1),
the automorphism X -> X^g, rescale by the last prime, the tensor product and
the NTT pair, on random rows of every prime.

Two rings: the toy ring N = 2^12 (digits of 2 primes) and the benchmark's
N = 2^16 ring (digits of 8 primes; there ModUp leaves each digit's own rows
out of its one forward transform and ModDown / rescale run as epilogues of the
two-pass transform, paths the toy ring does not take).  Levels are chosen so
that the last digit is ragged and the top level is covered."""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu

CASES = {
    "toy12": dict(modup=[20, 4, 23], moddown=[20, 4, 0], rescale=[23, 1], tensor=[7]),
    "fgb16": dict(modup=[12, 29], moddown=[12, 29], rescale=[12, 1], tensor=[5]),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def pair(request):
    from paper_2410_11184_amd import hs
    from oracle import ckks
    p = synthetic.preset(request.param)
    return request.param, hs.Context(p), ckks.Context(**p)


def _rows(o, idx, seed):
    rng = np.random.default_rng(seed)
    out = np.stack([rng.integers(0, o.primes[t], o.N, dtype=np.uint64) for t in idx])
    out[:, :4] = np.array([[o.primes[t] - 1] for t in idx], dtype=np.uint64)   # extreme residues
    return out


def test_ntt_pair(pair):
    name, g, o = pair
    lv = CASES[name]["modup"][0]
    x = _rows(o, range(lv + 1), 1)
    f = g.ring("ntt", x, lv)
    for i in range(lv + 1):
        assert np.array_equal(f[i], o.ntt(x[i], i)), i
    assert np.array_equal(g.ring("intt", f, lv), x)


def test_modup(pair):
    name, g, o = pair
    for lv in CASES[name]["modup"]:
        d = _rows(o, range(lv + 1), 10 + lv)
        got = g.ring("modup", d, lv)
        want = np.concatenate(o.mod_up(list(d), lv))
        assert got.shape == want.shape, (lv, got.shape, want.shape)
        bad = np.nonzero(~np.all(got == want, axis=1))[0]
        assert bad.size == 0, "level %d: rows %s differ" % (lv, bad[:8])


def test_moddown(pair):
    name, g, o = pair
    for lv in CASES[name]["moddown"]:
        idx = list(range(lv + 1)) + list(range(len(o.q), len(o.primes)))
        c = _rows(o, idx, 20 + lv)
        got = g.ring("moddown", c, lv)
        want = o.mod_down(list(c), lv)
        assert np.array_equal(got, want), lv


def test_automorphism(pair):
    name, g, o = pair
    lv = 6
    x = _rows(o, range(lv + 1), 3)
    for gal in (o.galois_rot(1, o.N), o.galois_rot(-77, o.N), 2 * o.N - 1):
        got = g.ring("auto", x, lv, gal)
        assert np.array_equal(got, x[:, o.automorph_perm(gal)]), gal


def test_rescale(pair):
    from oracle.ckks import Ciphertext
    name, g, o = pair
    for lv in CASES[name]["rescale"]:
        x = _rows(o, range(lv + 1), 30 + lv)
        got = g.ring("rescale", x, lv)
        want = o.rescale(Ciphertext([x], lv, 1.0)).c[0]
        assert np.array_equal(got, want), lv


def test_tensor(pair):
    from oracle.ckks import Ciphertext
    name, g, o = pair
    for lv in CASES[name]["tensor"]:
        a = [_rows(o, range(lv + 1), 40 + k) for k in range(4)]
        got = g.ring("tensor", np.concatenate(a), lv)
        d = o.tensor(Ciphertext(a[:2], lv, 1.0), Ciphertext(a[2:], lv, 1.0))
        assert np.array_equal(got, np.concatenate(d.c)), lv


def test_argument_errors(pair):
    from paper_2410_11184_amd import hs
    name, g, o = pair
    x = _rows(o, range(3), 5)
    with pytest.raises(hs.HSError) as e:
        g.ring("modup", x, 3)                      # 3 rows given, level 3 needs 4
    assert e.value.name == "HS_E_ARG"
    with pytest.raises(hs.HSError) as e:
        g.ring("auto", x, 2, 4)                    # even Galois element
    assert e.value.name == "HS_E_ARG"
    with pytest.raises(hs.HSError) as e:
        g.ring("rescale", x[:1], 0)
    assert e.value.name == "HS_E_LEVEL"
    with pytest.raises(hs.HSError) as e:
        g.ring("ntt", x, len(o.q) + 5)
    assert e.value.name == "HS_E_LEVEL"
