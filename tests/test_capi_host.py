"""CPU-side checks of the C ABI: the library loads, exports every function
declared in include/hs.h, and its host-only entry points (packing of
Section 4, parameter validation messages) behave; no GPU call is made."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "hs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hs_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2410_11184_amd import hs
    L = hs.lib()
    names = _declared()
    assert len(names) > 30
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert L.hs_version().decode().startswith("hs")


@pytest.mark.parametrize("m", [1, 4])
def test_pack_matches_oracle_layout(m):
    from paper_2410_11184_amd import hs
    from oracle import softmax as S
    slots, n = 1024, 64
    L = m * slots // n
    x = np.random.default_rng(m).uniform(-10, 0, (L, n))
    p = hs.pack_softmax(x, slots, 10.0)
    assert p.shape == (m, slots)
    assert np.array_equal(p, S.pack(x, m, slots))
    assert np.array_equal(hs.unpack_softmax(p, n), x)


def test_pack_range_check():
    from paper_2410_11184_amd import hs
    x = np.zeros((16, 64))
    x[2, 2] = -10.5
    with pytest.raises(hs.HSError) as e:
        hs.pack_softmax(x, 1024, 10.0)
    assert e.value.name == "HS_E_RANGE"
    with pytest.raises(hs.HSError) as e:
        hs.pack_softmax(np.zeros((8, 48)), 1024, 10.0)      # 8 x 64 padded slots < 1024
    assert e.value.name == "HS_E_ARG"


def test_pack_pads_a_dimension_that_is_not_a_power_of_two():
    from paper_2410_11184_amd import hs
    rng = np.random.default_rng(4)
    x = -10.0 * rng.random((32, 48))                       # 32 vectors, padded to 64 coordinates
    p = hs.pack_softmax(x, 1024, 10.0)
    assert p.shape == (2, 1024)                            # m = 32 * 64 / 1024 ciphertexts
    L, per = 32, 32
    for j in range(2):
        for c in range(per):
            coord = j * per + c
            want = x[:, coord] if coord < 48 else np.full(L, -10.0)
            assert np.array_equal(p[j, c * L:(c + 1) * L], want), (j, c)
    assert np.array_equal(hs.unpack_softmax(p, 48), x)


def test_last_error_is_thread_local_string():
    from paper_2410_11184_amd import hs
    L = hs.lib()
    st = L.hs_pack_softmax(np.zeros(9), 1, 9, 8, 1.0, None, ctypes.byref(ctypes.c_size_t()))
    assert st == -2
    assert b"n must be <= slots" in L.hs_last_error()


def test_tune_decisions_round_trip(tmp_path):
    # host-only: decisions are text; unknown kernels or choices are skipped
    from paper_2410_11184_amd import hs
    hs.tune_clear()
    f = tmp_path / "decisions.json"
    f.write_text('{"key": "conv N=4096 k=2 m=24 groups=8", "choice": "mfma", "us": {}}\n'
                 '{"key": "ntt N=65536 rows=13 groups=64 forward", "choice": "storage-order", "us": {}}\n'
                 '{"key": "ntt N=65536 rows=13 groups=64 inverse", "choice": "no-such-variant"}\n'
                 '{"key": "other N=1", "choice": "valu"}\n')
    assert hs.tune_load(f) == 2
    got = {r["key"]: r["choice"] for r in hs.tune_report()}
    assert got == {"conv N=4096 k=2 m=24 groups=8": "mfma", "ntt N=65536 rows=13 groups=64 forward": "storage-order"}
    g = tmp_path / "saved.json"
    hs.tune_save(g)
    hs.tune_clear()
    assert hs.tune_report() == []
    assert hs.tune_load(g) == 2
    hs.tune_clear()
    with pytest.raises(hs.HSError):
        hs.tune_load(tmp_path / "missing.json")


def test_prime_sizes_below_32_bits_refused():
    # the device reductions need primes of at least 32 bits; the check runs
    # before any device call, so it holds on a machine without a GPU
    from paper_2410_11184_amd import hs
    import synthetic
    p = dict(synthetic.preset("toy12"))
    p["q_bits"] = [31] + p["q_bits"][1:]
    with pytest.raises(hs.HSError) as e:
        hs.Context(p)
    assert e.value.name == "HS_E_PARAM"
    assert "32, 61" in str(e.value)


@pytest.mark.parametrize("case", [(0.98 / 256, 1.0001, 31, 0.5), (0.98 / 4096, 2.0, 15, 0.25),
                                  (0.01, 1.0, 7, 1.0), (0.5, 1.5, 3, 1 / 3), (0.98 / 256, 1.0, 63, 0.5),
                                  (0.5, 1.5, 31, 0.5)])
def test_minimax_coefficients_equal_the_oracle(case):
    # the library's normalisation polynomials (binary128 final solve) and the
    # oracle's (mpmath) follow one specification: the same doubles, also for
    # a near-exact fit (degree 31 on [0.5, 1.5]: error at the double's
    # rounding, the exchange stopped by its 2^-40 rule)
    from paper_2410_11184_amd import hs
    from oracle import polyeval as PE
    a, b, d, e = case
    assert np.array_equal(hs.minimax(a, b, d, e), np.array(PE.minimax_invpow(a, b, d, e)))
    with pytest.raises(hs.HSError):
        hs.minimax(b, a, d, e)
