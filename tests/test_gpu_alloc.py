"""Device memory through the caller's allocator (hs_ctx_create_ex; the
binding's default is torch's caching allocator): the results are the words
of a context on the library's own hipMalloc, every block handed out comes
back at hs_ctx_destroy, and an allocator that returns NULL gives HS_E_OOM
(during creation, and during key generation) with every block it did hand
out returned.  The failures are forced from the host (the callback declines);
no kernel sees a bad address."""
import gc

import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu


def _counting(fail_after=None):
    from paper_2410_11184_amd import hs

    class Counting(hs.TorchAllocator):
        def __init__(self):
            super().__init__(0)
            self.calls = 0
            self.fail_after = fail_after

        def get(self, nbytes, stream):
            self.calls += 1
            if self.fail_after is not None and self.calls > self.fail_after:
                return None
            return super().get(nbytes, stream)

    return Counting()


def _product(ctx):
    z = np.random.default_rng(3).uniform(-1, 1, ctx.slots)
    a = ctx.encrypt(z, 10, ctx.delta, 7)
    return ctx.rotate(ctx.mult(a, a), 3).export()


def test_same_words_and_everything_returned():
    from paper_2410_11184_amd import hs
    p = synthetic.preset("toy12")
    own = hs.Context(p, allocator=None)
    own.keygen(21)
    own.add_rotation_keys([3])
    want = _product(own)
    del own
    alloc = _counting()
    ctx = hs.Context(p, allocator=alloc)
    ctx.keygen(21)
    ctx.add_rotation_keys([3])
    got = _product(ctx)
    assert np.array_equal(got, want)
    assert alloc.calls > 0 and alloc.live
    del ctx
    gc.collect()
    assert alloc.live == {}, "blocks not returned: %d" % len(alloc.live)


@pytest.mark.parametrize("fail_after", [0, 1, 4, 9])
def test_creation_out_of_memory_returns_everything(fail_after):
    from paper_2410_11184_amd import hs
    alloc = _counting(fail_after)
    with pytest.raises(hs.HSError) as e:
        hs.Context(synthetic.preset("toy12"), allocator=alloc)
    assert e.value.name == "HS_E_OOM"
    assert alloc.calls >= fail_after + 1
    gc.collect()
    assert alloc.live == {}


def test_keygen_out_of_memory_returns_everything():
    from paper_2410_11184_amd import hs
    alloc = _counting()
    ctx = hs.Context(synthetic.preset("toy12"), allocator=alloc)
    alloc.fail_after = alloc.calls          # the arena's first chunk is declined
    with pytest.raises(hs.HSError) as e:
        ctx.keygen(5)
    assert e.value.name == "HS_E_OOM"
    ctx.close()            # (the exception's traceback still refers to ctx)
    assert alloc.live == {}


def test_both_callbacks_or_neither():
    import ctypes
    from paper_2410_11184_amd import hs
    p = synthetic.preset("toy12")
    alloc = _counting()
    qb = (ctypes.c_int * len(p["q_bits"]))(*p["q_bits"])
    pb = (ctypes.c_int * len(p["p_bits"]))(*p["p_bits"])
    prm = hs.hs_params(log_n=p["logN"], n_q=len(p["q_bits"]), q_bits=qb, n_p=len(p["p_bits"]), p_bits=pb,
                       digit=p["digit"], hamming=0, sigma=3.2, log_scale=p["log_scale"], user_top=p["user_top"])
    h = ctypes.c_void_p()
    st = hs.lib().hs_ctx_create_ex(ctypes.byref(prm), 0, None, alloc.alloc_cb, hs._FREE_FN(), None, ctypes.byref(h))
    assert hs.ERRORS[st] == "HS_E_ARG" and not h.value
